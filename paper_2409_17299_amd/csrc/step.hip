// step.hip -- the event-generator step on the GPU.
//
// One launch processes the leptons of one generation round (electrons, then
// positrons, as two source ranges) or a range of photons: Algorithm 1 for
// every particle; Algorithm 2 is the host loop over rounds in api.cpp.  A
// launch is three kernels:
//   count: every lane runs the sub-cycle loop of one particle, one sub-cycle
//          per loop trip; a lane whose particle reached the end of the step
//          takes the next one from a global queue (one atomic per wave), so
//          lanes stay busy while the event counts of particles differ -- the
//          role the paper's SortHandledParticles plays for a SIMD chunk
//          (Sec. 4.3).  It records each particle's event count and writes the
//          final state of particles without events.
//   scan:  exclusive prefix sum of the counts (single pass, decoupled
//          look-back between tiles) -> the append offset of every particle's
//          first child, and the list of particles with events.
//   write: re-runs the particles with events (same draws, same arithmetic)
//          and writes their children at the final offsets and their final
//          state.
// The append order therefore is: particles in index order, children of one
// particle in event order -- the same for every run and every grid size.

#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "lib.h"
#include "line_rule.h"
#include "physics.h"
#include "step.h"

namespace sfqed {

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// ------------------------------------------------------------------ look-back
// State word: [epoch:24][flag:2][value:38]; flag 1 = aggregate, 2 = inclusive prefix.
// Flag and value travel in one 64-bit word, so relaxed device-scope atomics
// suffice: no other data is published through it.  (Release/acquire at device
// scope would write back / invalidate the XCD-local L2 at every probe.)
constexpr uint64_t kValMask = (1ull << 38) - 1;

__device__ __forceinline__ void lb_publish(uint64_t* st, uint32_t epoch, uint64_t flag, uint64_t val) {
  const uint64_t v = ((uint64_t)epoch << 40) | (flag << 38) | (val > kValMask ? kValMask : val);
  __hip_atomic_store(st, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Run by all 64 lanes of one wave per tile.  Each probe reads the states of
// the 64 preceding tiles at once: the aggregates up to the nearest inclusive
// prefix are summed with a wave reduction, otherwise the window moves back by
// 64 tiles.  Returns the exclusive prefix of the tile (tile 0's is `base`).
__device__ int64_t lookback(uint64_t* st, int64_t tile, int64_t agg, int64_t base, uint32_t epoch) {
  const int lane = lane_id();
  if (tile == 0) {
    if (lane == 0) lb_publish(st, epoch, 2, (uint64_t)(base + agg));
    return base;
  }
  if (lane == 0) lb_publish(st + tile, epoch, 1, (uint64_t)agg);
  int64_t excl = 0;
  int64_t top = tile - 1;  // lane l probes tile top - l
  while (true) {
    const int64_t k = top - lane;
    uint64_t v = 0;
    bool ready = true;
    uint32_t fl = 2;  // tiles before the first one count as an empty prefix
    if (k >= 0) {
      v = __hip_atomic_load(st + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      fl = (uint32_t)((v >> 38) & 3);
      ready = (uint32_t)(v >> 40) == epoch && fl != 0;
    }
    if (!__all(ready)) {
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    const uint64_t pm = __ballot(fl == 2);
    const int stop = pm ? __builtin_ctzll(pm) : 63;
    int64_t val = (lane <= stop && k >= 0) ? (int64_t)(v & kValMask) : 0;
    for (int off = 32; off > 0; off >>= 1) val += __shfl_xor(val, off);
    excl += val;
    if (pm) break;
    top -= 64;
  }
  if (lane == 0) lb_publish(st + tile, epoch, 2, (uint64_t)(excl + agg));
  return excl;
}

// ------------------------------------------------------------------ per-lane choice of launch constants
// A launch may cover two source ranges, and an appended particle finds its
// fields through the species of its root, so a lane picks arrays at run time.
// An array of kernel arguments indexed per lane would be fetched with a global
// load from argument memory, a memory round trip in front of every access
// through the pointer, and keeping every candidate in scalar registers spills
// them; the kernels therefore copy the candidates into a small table in LDS
// when they start and a lane reads its entry from there.
// (SrcTable, in step.h, is that table.)

// a pointer from the table, known to address global memory
template <typename E>
__device__ __forceinline__ E* gptr(uint64_t v) {
  return (E*)reinterpret_cast<__attribute__((address_space(1))) E*>(v);
}

template <typename T>
__device__ __forceinline__ void fill_part(uint64_t* w, const SpeciesView<T>& s, const Rec<T>* rec, const T* pos,
                                          int64_t begin) {
  w[kPx] = (uint64_t)s.px;
  w[kPy] = (uint64_t)s.py;
  w[kPz] = (uint64_t)s.pz;
  w[kX] = (uint64_t)s.x;
  w[kY] = (uint64_t)s.y;
  w[kZ] = (uint64_t)s.z;
  w[kW] = (uint64_t)s.w;
  w[kTau] = (uint64_t)s.tau;
  w[kId] = (uint64_t)s.id;
  w[kAlive] = (uint64_t)s.alive;
  w[kNev] = (uint64_t)s.nev;
  w[kRec] = (uint64_t)rec;
  w[kPos] = (uint64_t)pos;
  w[kBegin] = (uint64_t)begin;
}
template <typename T>
__device__ __forceinline__ void fill_field(uint64_t* w, const FieldView<T>& f) {
  w[kEx] = (uint64_t)f.ex;
  w[kEy] = (uint64_t)f.ey;
  w[kEz] = (uint64_t)f.ez;
  w[kBx] = (uint64_t)f.bx;
  w[kBy] = (uint64_t)f.by;
  w[kBz] = (uint64_t)f.bz;
  w[kStride] = (uint64_t)f.stride;
  w[kFieldCount] = (uint64_t)f.n;
}

// one thread per entry (the caller synchronises the block afterwards)
template <typename T>
__device__ __forceinline__ void stage_sources(const StepArgs<T>& a, SrcTable* t) {
  switch (threadIdx.x) {
    case 0: fill_part<T>(t->part[0], a.src[0], a.src_rec[0], a.src_pos[0], a.begin[0]); break;
    case 1: fill_part<T>(t->part[1], a.src[1], a.src_rec[1], a.src_pos[1], a.begin[1]); break;
    case 2: fill_field<T>(t->field[0], a.f[0]); break;
    case 3: fill_field<T>(t->field[1], a.f[1]); break;
    case 4: fill_field<T>(t->field[2], a.f[2]); break;
    case 5:
      t->stats = (uint64_t)a.stats;
      t->pad = 0;
      break;
    default: break;
  }
}

// ------------------------------------------------------------------ particle state
template <typename T>
struct Lane {
  int64_t k;  // particle of the launch
  int64_t i;  // its index in the source of its part
  int32_t part;
  T p[3], x[3], E[3], B[3];
  double tau;
  T t, t0;
  uint64_t id;
  uint32_t root;
  float w;
  int32_t j;
  bool capped;
  bool changed;  // state differs from what was loaded
  T lz, lh;      // the last event's sampler value z and sub-interval h (logged by the count pass)
};

// E and B of the particle's root (children keep the fields of the particle
// they descend from; the fields are constant over the step).  A root that
// names no particle (species > 2 or an index past the species' fields: only a
// corrupted append record has one) gets no fields, so the particle has no
// events, and raises a statistics flag that the host reports as an error.
template <typename T>
__device__ __forceinline__ void load_fields(const SrcTable* src, uint32_t root, T (&E)[3], T (&B)[3]) {
  const uint32_t sp = root >> 30;
  const uint64_t* f = src->field[sp < 3 ? sp : 0];
  const int64_t idx = (int64_t)(root & 0x3FFFFFFFu);
  if (sp >= 3 || (f[kStride] && idx >= (int64_t)f[kFieldCount])) {
    atomicOr(gptr<unsigned long long>(src->stats) + kStatBadRoot, 1ull);
    E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = T(0);
    return;
  }
  const int64_t o = f[kStride] ? idx : 0;
  E[0] = gptr<const T>(f[kEx])[o];
  E[1] = gptr<const T>(f[kEy])[o];
  E[2] = gptr<const T>(f[kEz])[o];
  B[0] = gptr<const T>(f[kBx])[o];
  B[1] = gptr<const T>(f[kBy])[o];
  B[2] = gptr<const T>(f[kBz])[o];
}

// Issues the loads of the state of particle k of the launch; a particle of the
// input ensemble (kMain) also loads its fields (unless kFields is off), an
// appended particle finds them through its root afterwards.  Positions are
// zero unless they are tracked.
template <typename T, bool kMain, bool kFields = true>
__device__ __forceinline__ void load_state(const StepArgs<T>& a, const SrcTable* src, int64_t k, Lane<T>& L) {
  const bool p1 = k >= a.n0;
  const int part = p1 ? 1 : 0;
  const uint64_t* w = src->part[part];
  const int64_t i = (int64_t)w[kBegin] + (p1 ? k - a.n0 : k);
  L.k = k;
  L.i = i;
  L.part = part;
  L.j = 0;
  L.capped = false;
  L.changed = false;
  if constexpr (kMain) {
    // the root is the particle itself: its fields load together with its state
    L.root = ((uint32_t)(a.species + part) << 30) | (uint32_t)i;
    if constexpr (kFields) load_fields<T>(src, L.root, L.E, L.B);
    L.p[0] = gptr<const T>(w[kPx])[i];
    L.p[1] = gptr<const T>(w[kPy])[i];
    L.p[2] = gptr<const T>(w[kPz])[i];
    if (a.positions) {
      L.x[0] = gptr<const T>(w[kX])[i];
      L.x[1] = gptr<const T>(w[kY])[i];
      L.x[2] = gptr<const T>(w[kZ])[i];
    } else {
      L.x[0] = L.x[1] = L.x[2] = T(0);
    }
    L.tau = gptr<const double>(w[kTau])[i];
    L.id = gptr<const uint64_t>(w[kId])[i];
    L.w = gptr<const float>(w[kW])[i];
    L.t = T(0);
    L.t0 = T(0);
  } else {
    Rec<T> r;
    rec_load<T>(gptr<const Rec<T>>(w[kRec]), i, r);
    L.p[0] = r.px;
    L.p[1] = r.py;
    L.p[2] = r.pz;
    L.t = r.tb;
    L.t0 = r.tb;
    L.tau = r.tau;
    L.id = r.id;
    L.w = r.w;
    L.root = r.root;
    if (a.positions) {
      const T* q = gptr<const T>(w[kPos]) + 4 * i;
      L.x[0] = q[0];
      L.x[1] = q[1];
      L.x[2] = q[2];
    } else {
      L.x[0] = L.x[1] = L.x[2] = T(0);
    }
  }
}

template <typename T>
__device__ __forceinline__ void load_lane(const StepArgs<T>& a, const SrcTable* src, int64_t k, Lane<T>& L) {
  if (a.from_main) {
    load_state<T, true>(a, src, k, L);
  } else {
    load_state<T, false>(a, src, k, L);
    load_fields<T>(src, L.root, L.E, L.B);
  }
}

// What a lane stores: a child record, or its particle's final state (momentum
// when it changed, position, optical depth; for records also the event count
// and alive flag when asked) and, in the count kernel, the event count;
// staged in registers by the sub-cycle, stored by flush().
constexpr uint32_t kOutChild = 1u;     // r is a child record for the append buffer, at = its index
constexpr uint32_t kOutFinal = 2u;     // r holds the final state of particle `at` of its source
constexpr uint32_t kOutCount = 4u;     // the event count r.nev goes to counts[k] (and nev[at] of the source)
constexpr uint32_t kOutMomentum = 8u;  // the final state includes the momentum
constexpr uint32_t kOutDied = 16u;     // the particle was removed (photon at its event)
constexpr uint32_t kOutPart1 = 32u;    // the particle belongs to the second source range

template <typename T>
struct Outbox {
  Rec<T> r;
  T x[3];
  int64_t at;
  int64_t k;
  uint32_t what;
};

template <typename T>
__device__ __forceinline__ void stage_final(const StepArgs<T>& a, const Lane<T>& L, bool momentum, bool died,
                                            bool final_state, Outbox<T>& O) {
  O.r.px = L.p[0];
  O.r.py = L.p[1];
  O.r.pz = L.p[2];
  O.r.tb = L.t0;
  O.r.tau = L.tau;
  O.r.id = L.id;
  O.r.w = L.w;
  O.r.root = L.root;
  O.r.nev = L.j;
  O.r.alive = died ? 0u : 1u;
  O.x[0] = L.x[0];
  O.x[1] = L.x[1];
  O.x[2] = L.x[2];
  O.at = L.i;
  O.k = L.k;
  // W = 0 all along: nothing moved, nothing to store
  const bool store = final_state && (L.changed || died || (a.write_nev && !a.from_main));
  O.what |= (store ? kOutFinal : 0u) | (momentum ? kOutMomentum : 0u) | (died ? kOutDied : 0u) |
            (L.part ? kOutPart1 : 0u);
}

template <typename T>
__device__ __forceinline__ void flush(const StepArgs<T>& a, const SrcTable* src, Outbox<T>& O) {
  const uint32_t what = O.what;
  const uint64_t* w = src->part[(what & kOutPart1) ? 1 : 0];
  const int64_t i = O.at;
  if (what & kOutChild) {
    rec_store<T>(a.out_rec[0], i, O.r);
    if (a.positions) {
      T* q = a.out_pos[0] + 4 * i;
      q[0] = O.x[0];
      q[1] = O.x[1];
      q[2] = O.x[2];
      q[3] = T(0);
    }
  }
  if (what & kOutCount) {
    a.counts[O.k] = O.r.nev;
    if (a.from_main && w[kNev]) gptr<int32_t>(w[kNev])[i] = O.r.nev;
  }
  if (what & kOutFinal) {
    const bool momentum = (what & kOutMomentum) != 0, died = (what & kOutDied) != 0;
    if (a.from_main) {
      if (momentum) {
        gptr<T>(w[kPx])[i] = O.r.px;
        gptr<T>(w[kPy])[i] = O.r.py;
        gptr<T>(w[kPz])[i] = O.r.pz;
      }
      if (a.positions) {
        gptr<T>(w[kX])[i] = O.x[0];
        gptr<T>(w[kY])[i] = O.x[1];
        gptr<T>(w[kZ])[i] = O.x[2];
      }
      gptr<double>(w[kTau])[i] = O.r.tau;
      if (died) gptr<uint8_t>(w[kAlive])[i] = 0;
    } else {
      using C = RecChunks<T>;
      rec_store_part<T>(gptr<Rec<T>>(w[kRec]), i, O.r, momentum ? 0 : C::kTau,
                        (a.write_nev || died) ? C::kCount : C::kTail);
      if (a.positions) {
        T* q = gptr<T>(w[kPos]) + 4 * i;
        q[0] = O.x[0];
        q[1] = O.x[1];
        q[2] = O.x[2];
      }
    }
  }
  O.what = 0;
}

// Final state of a processed photon, stored at once.
template <typename T>
__device__ __forceinline__ void store_final(const StepArgs<T>& a, const SrcTable* src, const Lane<T>& L,
                                            bool momentum, bool died) {
  Outbox<T> O;
  O.what = 0;
  stage_final<T>(a, L, momentum, died, true, O);
  flush<T>(a, src, O);
}

// Tables as the kernels see them: FP32 tables staged in LDS, FP64 in HBM.
struct LdsTables {
  const SrcTable* src;
  const float2* herm;
  const float* cdf;
};

template <typename T>
__device__ __forceinline__ T rate_of(const StepArgs<T>& a, const LdsTables& lt, int process, T chi, T s_chi,
                                     T energy) {
  if constexpr (sizeof(T) == 4) {
    const RateView& r = a.tab.rate[process];
    return process == 0 ? rate_rad32_s(lt.herm, r.n, r.hs_lo, r.inv_h, chi, s_chi, energy)
                        : rate_pair32_s(lt.herm, r.n, r.hs_lo, r.inv_h, chi, s_chi, energy);
  } else {
    return process == 0 ? rate_rad64(a.tab.rate[0], chi, energy) : rate_pair64(a.tab.rate[1], chi, energy);
  }
}

// s_chi = ln chi (used by the FP32 path only)
template <typename T>
__device__ __forceinline__ void sample_of(const StepArgs<T>& a, const LdsTables& lt, int process, T chi, T s_chi,
                                          uint32_t k, T& v, T& omv) {
  if constexpr (sizeof(T) == 4) {
    if (process == 0) sample_rad32_s(lt.cdf, a.tab.cdf[0], chi, s_chi, k, v, omv);
    else sample_pair32_s(lt.cdf, a.tab.cdf[1], s_chi, k, v, omv);
  } else {
    if (process == 0) sample_rad64(a.tab.cdf[0], chi, k, v, omv);
    else sample_pair64(a.tab.cdf[1], chi, k, v, omv);
  }
}

// The emission sampler split at its last step: z = logit(delta) from the
// grids, then delta = sigmoid(z) and 1 - delta = sigmoid(-z).  The count pass
// logs z, so the write pass replays the event without the grids.
template <typename T>
__device__ __forceinline__ T sample_rad_z(const StepArgs<T>& a, const LdsTables& lt, T chi, T s_chi, uint32_t k) {
  if constexpr (sizeof(T) == 4) return sample_rad32_z(lt.cdf, a.tab.cdf[0], chi, s_chi, k);
  else return sample_rad64_z(a.tab.cdf[0], chi, k);
}
template <typename T>
__device__ __forceinline__ void sigmoid_of(T z, T& p, T& q) {
  if constexpr (sizeof(T) == 4) sigmoid_pair32(z, p, q);
  else sigmoid_pair64(z, p, q);
}

// ln chi for the FP32 path (the FP64 path takes its logarithms inside)
template <typename T>
__device__ __forceinline__ T log_chi(T chi) {
  if constexpr (sizeof(T) == 4) return chi > 0.f ? logf(chi) : 0.f;
  else return T(0);
}

// a / b: the hardware reciprocal on the FP32 path, IEEE division on the FP64 path
template <typename T>
__device__ __forceinline__ T quot(T a, T b) {
  if constexpr (sizeof(T) == 4) return a * __builtin_amdgcn_rcpf(b);
  else return a / b;
}

template <typename T>
__device__ __forceinline__ void advance_lepton(const StepArgs<T>& a, Lane<T>& L, T q, T h) {
  if (a.push) boris<T>(L.p, q, L.E, L.B, h);
  if (a.positions) {
    const T gi = T(1) / sqrt(T(1) + L.p[0] * L.p[0] + L.p[1] * L.p[1] + L.p[2] * L.p[2]);
    L.x[0] += L.p[0] * gi * h;
    L.x[1] += L.p[1] * gi * h;
    L.x[2] += L.p[2] * gi * h;
  }
}

template <typename T>
__device__ __forceinline__ void write_child(Rec<T>* out, T* pos, int64_t idx, const T p[3], const T x[3],
                                            bool positions, float w, double tau, uint64_t id, uint32_t root, T tb) {
  Rec<T> r;
  r.px = p[0];
  r.py = p[1];
  r.pz = p[2];
  r.tb = tb;
  r.tau = tau;
  r.id = id;
  r.w = w;
  r.root = root;
  r.nev = 0;
  r.alive = 1u;
  rec_store<T>(out, idx, r);
  if (positions) {
    T* q = pos + 4 * idx;
    q[0] = x[0];
    q[1] = x[1];
    q[2] = x[2];
    q[3] = T(0);
  }
}

// One sub-cycle of Algorithm 1 for a lepton.  Returns true when the particle
// has reached the end of the step.  kLog keeps what the write pass needs to
// replay an event in L.lz and L.lh.
template <typename T, bool kWrite, bool kLog = false>
__device__ __forceinline__ bool lepton_iter(const StepArgs<T>& a, const LdsTables& lt, Lane<T>& L, T q,
                                            int64_t out_base, Outbox<T>& O) {
  const T dtT = (T)a.dt;
  if (!(L.t < dtT)) return true;
  const T g = sqrt(T(1) + L.p[0] * L.p[0] + L.p[1] * L.p[1] + L.p[2] * L.p[2]);
  T W = T(0);
  const T chi0 = chi_of<T>(L.p, g, L.E, L.B);
  const T s0 = log_chi<T>(chi0);
  if (a.emission && !L.capped && (double)g >= a.gamma_min) W = rate_of<T>(a, lt, 0, chi0, s0, g);
  const T rem = dtT - L.t;
  const double X = (double)W * (double)rem;
  if (!(W > T(0)) || L.tau > X) {  // no event before the end of the step
    L.tau -= X;
    advance_lepton<T>(a, L, q, rem);
    L.t = dtT;
    L.changed |= X > 0.0 || a.push || a.positions;
    return true;
  }
  T h = quot<T>((T)L.tau, W);  // the optical depth runs out after h
  if (h > rem) h = rem;
  advance_lepton<T>(a, L, q, h);
  L.t += h;
  const uint4 u = draw(a.seed, L.id, a.step, (uint32_t)L.j);
  T chi_e = chi0, s_e = s0;  // the particle as it is at the event (unchanged unless pushed)
  if (a.push) {
    const T g2 = sqrt(T(1) + L.p[0] * L.p[0] + L.p[1] * L.p[1] + L.p[2] * L.p[2]);
    chi_e = chi_of<T>(L.p, g2, L.E, L.B);
    s_e = log_chi<T>(chi_e);
  }
  const T z = sample_rad_z<T>(a, lt, chi_e, s_e, u.x);
  T d, omd;
  sigmoid_of<T>(z, d, omd);
  if constexpr (kLog) {
    L.lz = z;
    L.lh = h;
  }
  if (kWrite) {
    const int64_t o = out_base + L.j;
    if (o < a.out_cap) {  // the photon: k = delta p, born here
      const uint4 v = draw(a.seed, L.id, a.step, (uint32_t)L.j | 0x80000000u);
      O.r.px = d * L.p[0];
      O.r.py = d * L.p[1];
      O.r.pz = d * L.p[2];
      O.r.tb = L.t;
      O.r.tau = exp_depth_t<T>(u.z);
      O.r.id = (uint64_t)v.x | ((uint64_t)v.y << 32);
      O.r.w = L.w;
      O.r.root = L.root;
      O.r.nev = 0;
      O.r.alive = 1u;
      O.x[0] = L.x[0];
      O.x[1] = L.x[1];
      O.x[2] = L.x[2];
      O.at = o;
      O.what = kOutChild;
    }
  }
  L.p[0] *= omd;  // collinear recoil: photon k = delta p, lepton (1 - delta) p
  L.p[1] *= omd;
  L.p[2] *= omd;
  L.tau = exp_depth_t<T>(u.y);
  L.changed = true;
  ++L.j;
  if (L.j >= a.max_events) L.capped = true;
  return false;
}

// The photon counterpart: pair rate, straight-line motion, removed at its
// first event (the pair takes xi and 1 - xi of its momentum).
template <typename T, bool kWrite>
__device__ __forceinline__ bool photon_iter(const StepArgs<T>& a, const LdsTables& lt, Lane<T>& L,
                                            int64_t out_base) {
  const T dtT = (T)a.dt;
  if (!(L.t < dtT)) return true;
  T eps, chi0;
  const bool can_pair = photon_chi<T>(L.p, L.E, L.B, eps, chi0);
  T W = T(0);
  const T s0 = log_chi<T>(chi0);
  if (a.pair && can_pair) W = rate_of<T>(a, lt, 1, chi0, s0, eps);
  const T rem = dtT - L.t;
  const double X = (double)W * (double)rem;
  const T inv_eps = eps > T(0) ? T(1) / eps : T(0);
  if (!(W > T(0)) || L.tau > X) {
    L.tau -= X;
    if (a.positions) {
      L.x[0] += L.p[0] * inv_eps * rem;
      L.x[1] += L.p[1] * inv_eps * rem;
      L.x[2] += L.p[2] * inv_eps * rem;
    }
    L.t = dtT;
    L.changed |= X > 0.0 || a.positions;
    return true;
  }
  T h = quot<T>((T)L.tau, W);
  if (h > rem) h = rem;
  if (a.positions) {
    L.x[0] += L.p[0] * inv_eps * h;
    L.x[1] += L.p[1] * inv_eps * h;
    L.x[2] += L.p[2] * inv_eps * h;
  }
  L.t += h;
  if (kWrite) {
    const uint4 u = draw(a.seed, L.id, a.step, 0u);
    T xi, omx;
    sample_of<T>(a, lt, 1, chi0, s0, u.x, xi, omx);
    const int64_t o = out_base;
    if (o < a.out_cap) {
      const uint4 v = draw(a.seed, L.id, a.step, 0x80000000u);
      const T pe[3] = {xi * L.p[0], xi * L.p[1], xi * L.p[2]};
      const T pp[3] = {omx * L.p[0], omx * L.p[1], omx * L.p[2]};
      write_child<T>(a.out_rec[0], a.out_pos[0], o, pe, L.x, a.positions, L.w, exp_depth_t<T>(u.z),
                     (uint64_t)v.x | ((uint64_t)v.y << 32), L.root, L.t);
      write_child<T>(a.out_rec[1], a.out_pos[1], o, pp, L.x, a.positions, L.w, exp_depth_t<T>(u.w),
                     (uint64_t)v.z | ((uint64_t)v.w << 32), L.root, L.t);
    }
  }
  L.j = 1;
  L.changed = true;
  return true;
}

template <typename T, bool kPhoton>
__device__ __forceinline__ LdsTables stage_tables(const StepArgs<T>& a, float* lds) {
  SrcTable* src = reinterpret_cast<SrcTable*>(lds);
  stage_sources<T>(a, src);
  lds += sizeof(SrcTable) / sizeof(float);
  LdsTables lt{src, nullptr, nullptr};
  if constexpr (sizeof(T) == 4) {
    const int p = kPhoton ? 1 : 0;
    const RateView& r = a.tab.rate[p];
    const CdfView& c = a.tab.cdf[p];
    float2* h = reinterpret_cast<float2*>(lds);
    float* cdf = lds + 2 * r.n;
    for (int i = threadIdx.x; i < r.n; i += blockDim.x) h[i] = r.herm[i];
    const int nc = c.rows32 * c.cols32;
    for (int i = threadIdx.x; i < nc; i += blockDim.x) cdf[i] = c.f32[i];
    lt.herm = h;
    lt.cdf = cdf;
  }
  __syncthreads();
  return lt;
}

// ------------------------------------------------------------------ work distribution
// Lepton kernels: lanes whose particle has finished take the next one from a
// queue held by their wave; the wave refills that queue in chunks from a
// counter.  The particles of the launch are split into kQueueParts contiguous
// ranges, each with its own counter on its own cache line.  A wave starts on
// the range of its XCD (work-groups are dealt to the eight XCDs in turn) and
// moves on to the following ranges once that one is used up.  Device-scope
// atomics that every wave of the chip sends to one address serialise at the
// memory side; eight lines and chunks of about remaining / (2 waves of the
// range), between kChunkMin and kChunkMax, keep that cost small, and the
// chunks shrink towards the end so the tail stays balanced.
struct WaveQueue {
  uint64_t next, end;  // wave-uniform
  uint32_t part, tried;
  bool done;
};

__device__ __forceinline__ void wq_init(WaveQueue& q) {
  q.next = q.end = 0;
  q.part = blockIdx.x % kQueueParts;
  q.tried = 0;
  q.done = false;
}

// Returns the item index of this lane (>= n: none) for lanes with need set.
// ctr: kQueueParts counters, kQueueStride words apart, zero at launch.
// kOneChunk: serve the lanes from one contiguous range only (lanes left over
// wait for the next call), so that the lanes served get consecutive items in
// lane order -- what the event log's records assume.
template <bool kOneChunk = false>
__device__ __forceinline__ uint64_t wq_take(WaveQueue& q, bool need, uint64_t n, unsigned long long* ctr,
                                            uint32_t waves) {
  uint64_t m = __ballot(need);
  uint64_t got = ~0ull;
  const uint64_t waves_part = waves / kQueueParts > 0 ? waves / kQueueParts : 1;
  while (m && !q.done) {
    const uint64_t avail = q.end - q.next;
    if (avail == 0) {
      const uint64_t lo = n * q.part / kQueueParts, hi = n * (q.part + 1) / kQueueParts, len = hi - lo;
      unsigned long long* c = ctr + (size_t)q.part * kQueueStride;
      uint64_t base = 0;
      uint64_t chunk = kChunkMin;
      if (lane_id() == 0) {
        const uint64_t seen = __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t rem = seen < len ? len - seen : 0;
        chunk = rem / (2ull * waves_part);
        chunk = chunk < kChunkMin ? kChunkMin : (chunk > kChunkMax ? kChunkMax : chunk);
        base = seen < len ? atomicAdd(c, (unsigned long long)chunk) : len;
      }
      base = readlane64(base, 0);
      chunk = readlane64(chunk, 0);
      if (base >= len) {  // this range is used up: go on to the next one
        if (++q.tried == kQueueParts) {
          q.done = true;
          break;
        }
        q.part = (q.part + 1) % kQueueParts;
        continue;
      }
      q.next = lo + base;
      q.end = base + chunk < len ? lo + base + chunk : hi;
      continue;
    }
    const uint32_t cnt = (uint32_t)__popcll(m);
    const uint32_t take = (uint64_t)cnt < avail ? cnt : (uint32_t)avail;
    const uint32_t r = mbcnt(m);
    if (((m >> lane_id()) & 1ull) && r < take) got = q.next + r;
    // lanes served drop out of the mask
    uint64_t served = 0;
    {
      const uint64_t mine = (((m >> lane_id()) & 1ull) && r < take) ? 1ull : 0ull;
      served = __ballot(mine != 0);
    }
    m &= ~served;
    q.next += take;
    if constexpr (kOneChunk) break;
  }
  return got;
}

// ------------------------------------------------------------------ event log
// With the log on, the lepton count pass records what the write pass needs
// to replay each event without the tables (format in event_log.h): per trip
// of a wave in which some lane had an event, or finished a particle that had
// one, a record of the lanes that took a new particle (and the launch index
// the first of them took) and of the lanes with an event, and per such lane
// a slot: the event's sampler value z = logit(delta) and sub-interval h, or
// the finished particle's optical depth.  A particle without events is never
// replayed.  When the pool runs out, the wave stops writing, raises the
// overflow flag and the direct write kernel does the launch's writes; every
// wave still adds up the bytes it would have needed, so that the host can
// grow the pool.
// Wave-uniform state of one wave's log, kept in 32-bit words (scalar
// registers are scarce in the count kernel).
struct LogWriter {
  uint32_t blk;   // current block (index in the pool, in units of kLogBlock)
  uint32_t pos;   // next record position in the block
  uint32_t recs;  // records of this wave, written or not
  uint32_t state; // 0: no block yet, 1: writing, 2: the pool ran out
};

// A lane's slot of a record (FP32: 8 bytes; FP64: 16).
template <typename T>
using LogSlot = typename std::conditional<sizeof(T) == 4, uint2, uint4>::type;

template <typename T>
__device__ __forceinline__ LogSlot<T> log_event_slot(T z, T h) {
  if constexpr (sizeof(T) == 4) {
    return make_uint2(fbits(z), fbits(h));
  } else {
    const uint64_t zb = __builtin_bit_cast(uint64_t, z), hb = __builtin_bit_cast(uint64_t, h);
    return make_uint4(lo32(zb), hi32(zb), lo32(hb), hi32(hb));
  }
}

template <typename T>
__device__ __forceinline__ LogSlot<T> log_final_slot(double tau) {
  const uint64_t b = __builtin_bit_cast(uint64_t, tau);
  if constexpr (sizeof(T) == 4) return make_uint2(lo32(b), hi32(b));
  else return make_uint4(lo32(b), hi32(b), 0u, 0u);
}

__device__ __forceinline__ void log_header(char* at, uint64_t w0, uint64_t w1, uint64_t w2, uint64_t tag) {
  uint4* h = reinterpret_cast<uint4*>(at);
  h[0] = make_uint4(lo32(w0), hi32(w0), lo32(w1), hi32(w1));
  h[1] = make_uint4(lo32(w2), hi32(w2), lo32(tag), hi32(tag));
}

// One trip of the wave: ev, the lane had an event; fin_with_events, its
// particle, which had events, finished; fresh, it took a new particle at the
// start of the trip (its launch index in L.k).
template <typename T>
__device__ __forceinline__ void log_trip(const StepArgs<T>& a, LogWriter& w, uint32_t wave, bool ev,
                                         bool fin_with_events, bool fresh, const Lane<T>& L) {
  constexpr uint32_t S = log_slot_bytes<T>();
  constexpr uint64_t R = log_record_bytes(S);
  constexpr uint32_t kPer = (uint32_t)log_records_per_block(S);
  const uint64_t m_part = __ballot(ev || fin_with_events);
  if (!m_part) return;
  const uint64_t m_fresh = __ballot(fresh), m_ev = __ballot(ev);
  w.recs += 1;
  if (w.state == 2) return;
  const int lane = lane_id();
  if (w.state == 0 || w.pos + 1 >= kPer) {  // the block's last position is kept for a marker
    uint32_t b = 0;
    if (lane == 0) b = (uint32_t)(atomicAdd(a.log_ctl + kLogUsed, 1ull));
    b = (uint32_t)__builtin_amdgcn_readfirstlane((int)b);
    const uint64_t blk = (uint64_t)b * kLogBlock;
    if (blk + kLogBlock > a.log_cap) {
      if (lane == 0) atomicOr(a.log_ctl + kLogOverflow, 1ull);
      w.state = 2;
      return;
    }
    if (lane == 0) {
      if (w.state == 1) log_header(a.log_pool + (uint64_t)w.blk * kLogBlock + (uint64_t)w.pos * R, 0, 0, blk, kLogJump);
      else a.log_head[wave] = blk + 1;
    }
    w.state = 1;
    w.blk = b;
    w.pos = 0;
  }
  // fresh lanes took consecutive launch indices in lane order (one queue range per trip)
  const uint64_t base = m_fresh ? readlane64((uint64_t)L.k, __builtin_ctzll(m_fresh)) : 0ull;
  char* rec = a.log_pool + (uint64_t)w.blk * kLogBlock + (uint64_t)w.pos * R;
  if (lane == 0) log_header(rec, m_fresh, m_ev, base, kLogRecord);
  if (ev || fin_with_events)
    *reinterpret_cast<LogSlot<T>*>(rec + kLogHeader + (uint64_t)S * lane) =
        ev ? log_event_slot<T>(L.lz, L.lh) : log_final_slot<T>(L.tau);
  w.pos += 1;
}

template <typename T>
__device__ __forceinline__ void log_close(const StepArgs<T>& a, const LogWriter& w, uint32_t wave) {
  constexpr uint64_t R = log_record_bytes(log_slot_bytes<T>());
  constexpr uint64_t kPer = log_records_per_block(log_slot_bytes<T>());
  if (lane_id() != 0) return;
  if (w.state == 0) a.log_head[wave] = 0;
  else if (w.state == 1) log_header(a.log_pool + (uint64_t)w.blk * kLogBlock + (uint64_t)w.pos * R, 0, 0, 0, kLogEnd);
  // the blocks this wave's records take (each block keeps its last position
  // for a marker), plus one for the end marker
  if (w.recs) atomicAdd(a.log_ctl + kLogNeed, (unsigned long long)(w.recs / (kPer - 1) + 2) * kLogBlock);
}

// ------------------------------------------------------------------ count kernels
// Leptons: event counts vary from 0 to hundreds, so lanes refill.
// A particle of the input ensemble (kMain) has its fields at its own index;
// an appended one finds them through its root, a second load after its record.
// kLog: the pass also writes the event log (above).
template <typename T, bool kMain, bool kLog>
__global__ void __launch_bounds__(kStepThreads, sizeof(T) == 4 ? kStepWavesPerSimd : 1) k_count_lepton(StepArgs<T> a) {
  extern __shared__ float lds[];
  const LdsTables lt = stage_tables<T, false>(a, lds);
  const uint64_t n = (uint64_t)a.n;
  const uint32_t waves = gridDim.x * (kStepThreads / 64);
  const uint32_t wave = blockIdx.x * (kStepThreads / 64) + (threadIdx.x >> 6);
  WaveQueue wq;
  wq_init(wq);
  Lane<T> L;
  Outbox<T> O;
  O.what = 0;
  LogWriter lw;
  lw.blk = lw.pos = lw.recs = lw.state = 0;
  T q = T(-1);
  bool have = false;
  int32_t local_max = 0;
  bool capped = false;
  while (true) {
    const uint64_t k = wq_take<kLog>(wq, !have, n, a.queue, waves);
    bool fresh = false;
    if (!have && k < n) {
      load_state<T, kMain>(a, lt.src, (int64_t)k, L);
      if (!kMain) load_fields<T>(lt.src, L.root, L.E, L.B);
      q = a.species + L.part == 0 ? T(-1) : T(1);
      have = true;
      fresh = true;
    }
    if (!__any(have)) break;
    bool fin = false;
    if (have) {
      fin = lepton_iter<T, false, kLog>(a, lt, L, q, 0, O);
      if (fin) {
        O.what = kOutCount;
        stage_final<T>(a, L, a.push != 0, false, L.j == 0, O);
        flush<T>(a, lt.src, O);
        local_max = L.j > local_max ? L.j : local_max;
        capped |= L.capped;
      }
    }
    if constexpr (kLog) log_trip<T>(a, lw, wave, have && !fin, have && fin && L.j > 0, fresh, L);
    if (fin) have = false;
  }
  if constexpr (kLog) log_close<T>(a, lw, wave);
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(local_max, off);
    local_max = o > local_max ? o : local_max;
  }
  if (lane_id() == 0 && local_max > 0) atomicMax(&a.stats[kStatMaxEvents], (unsigned long long)local_max);
  if (__any(capped) && lane_id() == 0) atomicOr(&a.stats[kStatCapped], 1ull);
}

// Photons: at most one event each; one photon per thread.
template <typename T>
__global__ void __launch_bounds__(kStepThreads, sizeof(T) == 4 ? kStepWavesPerSimd : 1) k_count_photon(StepArgs<T> a) {
  extern __shared__ float lds[];
  const LdsTables lt = stage_tables<T, true>(a, lds);
  int32_t any_event = 0;
  for (int64_t k = (int64_t)blockIdx.x * kStepThreads + threadIdx.x; k < a.n;
       k += (int64_t)gridDim.x * kStepThreads) {
    Lane<T> L;
    load_lane<T>(a, lt.src, k, L);
    if (a.from_main && a.src[0].alive[L.i] == 0) {  // a photon removed earlier is not processed
      a.counts[k] = 0;
      continue;
    }
    photon_iter<T, false>(a, lt, L, 0);
    a.counts[k] = L.j;
    if (a.from_main && a.src[0].nev) a.src[0].nev[L.i] = L.j;
    if (L.j == 0) store_final<T>(a, lt.src, L, false, false);
    any_event |= L.j;
  }
  if (__any(any_event) && lane_id() == 0) atomicMax(&a.stats[kStatMaxEvents], 1ull);
}

// The photon count pass of an appended range with the merge folded in: tiles
// of kMergedTile photons (kMergedItems per thread, item-major so that loads of
// one item are coalesced) are taken in order from a counter.  A photon without
// a pair event survives the step and is written, in its final state, straight
// into the main photon arrays at (photons there before the launch) +
// (survivors before it), the place the merge would give it.  A photon has at
// most one event, so the same count also places the others: a photon with an
// event is the (k - survivors before k)-th event of the launch, and its pair
// goes to the lepton buffers at the pair cursor plus that index.  This pass
// therefore writes the event list and first-child offsets itself (no counts,
// no scan).  A single-pass look-back over tiles gives the survivors before each
// tile; tiles are taken in order, so a block only waits for tiles that running
// blocks hold.  Every block reads the two cursors before it takes its first
// tile: the last tile, which moves them, cannot finish before every earlier
// tile has published, and a block that has not taken a tile holds one of them.
template <typename T>
__global__ void __launch_bounds__(kStepThreads, sizeof(T) == 4 ? kStepWavesPerSimd : 1)
    k_count_photon_merged(StepArgs<T> a) {
  extern __shared__ float lds[];
  const LdsTables lt = stage_tables<T, true>(a, lds);
  __shared__ int32_t wsum[kMergedItems][kStepThreads / 64];
  __shared__ int64_t s_tile, s_base;
  int64_t n = a.n;
  if (a.n_dev) {  // the range as the round's lepton launch left it
    const int64_t hi = *a.n_dev < a.n_cap ? *a.n_dev : a.n_cap;
    n = hi > a.n_base ? hi - a.n_base : 0;
  }
  const int64_t num_tiles = (n + kMergedTile - 1) / kMergedTile;
  if (num_tiles == 0) {  // an empty range: no events (the write kernel reads the list's length)
    if (blockIdx.x == 0 && threadIdx.x == 0) *const_cast<int64_t*>(a.list_len) = 0;
    return;
  }
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t dst0 = *a.dst_cursor, pair0 = *a.pair_cursor;
  int32_t any_event = 0;
  while (true) {
    __syncthreads();  // the previous tile's readers of s_tile, s_base and wsum are done
    if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(a.dst_ticket, 1ull);
    __syncthreads();
    const int64_t tile = s_tile;
    if (tile >= num_tiles) break;
    T p[kMergedItems][3], x[kMergedItems][3];
    double tau[kMergedItems];
    float w[kMergedItems];
    uint64_t id[kMergedItems];
    uint32_t surv = 0, event = 0;
#pragma unroll
    for (int it = 0; it < kMergedItems; ++it) {
      const int64_t k = tile * kMergedTile + (int64_t)it * kStepThreads + threadIdx.x;
      if (k < n) {
        Lane<T> L;
        load_lane<T>(a, lt.src, k, L);
        photon_iter<T, false>(a, lt, L, 0);
        any_event |= L.j;
        event |= (L.j != 0 ? 1u : 0u) << it;
        if (L.j == 0) {
          surv |= 1u << it;
          for (int c = 0; c < 3; ++c) {
            p[it][c] = L.p[c];
            x[it][c] = L.x[c];
          }
          tau[it] = L.tau;
          w[it] = L.w;
          id[it] = L.id;
        }
      }
    }
    uint64_t m[kMergedItems];
#pragma unroll
    for (int it = 0; it < kMergedItems; ++it) {
      m[it] = __ballot((surv >> it) & 1u);
      if (lane == 0) wsum[it][wave] = __popcll(m[it]);
    }
    __syncthreads();
    int32_t pre[kMergedItems];
    int32_t total = 0;
#pragma unroll
    for (int it = 0; it < kMergedItems; ++it) {
      int32_t before = 0, all = 0;
      for (int wv = 0; wv < kStepThreads / 64; ++wv) {
        before += wv < wave ? wsum[it][wv] : 0;
        all += wsum[it][wv];
      }
      pre[it] = total + before + (int32_t)mbcnt(m[it]);
      total += all;
    }
    if (wave == 0) {  // survivors of this launch before the tile
      const int64_t b = lookback(a.dst_state, tile, total, 0, a.dst_epoch);
      if (lane == 0) {
        s_base = b;
        if (tile == num_tiles - 1) {
          const int64_t events = n - (b + total);
          *a.dst_cursor = dst0 + b + total;
          *a.pair_cursor = pair0 + events;
          // a control word the scan writes in other launches; events past the
          // list's capacity make pairs past the lepton capacity, an overflow
          // the host reports, and are not written
          *const_cast<int64_t*>(a.list_len) = events < a.list_cap ? events : a.list_cap;
          atomicAdd(&a.stats[kStatEventParticles + 1], (unsigned long long)events);
        }
      }
    }
    __syncthreads();
    const SpeciesView<T>& d = a.dst;
#pragma unroll
    for (int it = 0; it < kMergedItems; ++it) {
      if ((event >> it) & 1u) {  // the e-th event of the launch, e = k - survivors before k
        const int64_t k = tile * kMergedTile + (int64_t)it * kStepThreads + threadIdx.x;
        const int64_t e = k - (s_base + pre[it]);
        if (e < a.list_cap) {
          a.list[e] = (int32_t)k;
          a.offsets[e] = pair0 + e;
        }
      }
      if (!((surv >> it) & 1u)) continue;
      const int64_t o = dst0 + s_base + pre[it];
      if (o >= a.dst_cap) continue;
      d.px[o] = p[it][0];
      d.py[o] = p[it][1];
      d.pz[o] = p[it][2];
      if (a.positions) {
        d.x[o] = x[it][0];
        d.y[o] = x[it][1];
        d.z[o] = x[it][2];
      }
      d.w[o] = w[it];
      d.tau[o] = tau[it];
      d.id[o] = id[it];
      d.alive[o] = 1;
    }
  }
  if (__any(any_event) && lane_id() == 0) atomicMax(&a.stats[kStatMaxEvents], 1ull);
}

// ------------------------------------------------------------------ scan kernel
// One tile of kScanTile counts per block: thread t holds items
// [16 t, 16 t + 16) of the tile (loaded as four 16-byte vectors when the tile
// is full).  The tile's event particles and their first child offsets are
// compacted into LDS relative to the tile while the two look-backs (children
// on wave 0, event particles on wave 1) run, then written out by the whole
// block, consecutive threads to consecutive entries.
__global__ void __launch_bounds__(kScanThreads) k_scan(ScanArgs s) {
  __shared__ int64_t sc[kScanThreads / 64];
  __shared__ int32_t sf[kScanThreads / 64];
  __shared__ int64_t s_tile, s_base_c, s_base_f;
  __shared__ int64_t l_off[kScanTile];
  __shared__ int32_t l_idx[kScanTile];
  const int tid = threadIdx.x;
  if (tid == 0) s_tile = (int64_t)atomicAdd(s.ticket, 1ull);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t k0 = tile * kScanTile + (int64_t)tid * kScanItems;
  int32_t c[kScanItems];
  if (k0 + kScanItems <= s.n) {
    const int4* v = reinterpret_cast<const int4*>(s.counts + k0);
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q) {
      const int4 x = v[q];
      c[4 * q] = x.x;
      c[4 * q + 1] = x.y;
      c[4 * q + 2] = x.z;
      c[4 * q + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) c[i] = k0 + i < s.n ? s.counts[k0 + i] : 0;
  }
  int64_t my_c = 0;
  int32_t my_f = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    my_c += c[i];
    my_f += c[i] > 0;
  }
  // wave-inclusive scans
  int64_t ic = my_c;
  int32_t inf = my_f;
  const int lane = lane_id();
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t oc = __shfl_up(ic, off);
    const int32_t of = __shfl_up(inf, off);
    if (lane >= off) {
      ic += oc;
      inf += of;
    }
  }
  const int wave = tid >> 6;
  if (lane == 63) {
    sc[wave] = ic;
    sf[wave] = inf;
  }
  __syncthreads();
  int64_t pre_c = 0, acc_c = 0;
  int32_t pre_f = 0, acc_f = 0;
  for (int wv = 0; wv < kScanThreads / 64; ++wv) {
    pre_c += wv < wave ? sc[wv] : 0;
    pre_f += wv < wave ? sf[wv] : 0;
    acc_c += sc[wv];
    acc_f += sf[wv];
  }
  // the tile's event particles, compacted relative to the tile
  int64_t lc = pre_c + ic - my_c;
  int32_t lf = pre_f + inf - my_f;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (c[i] > 0) {
      l_idx[lf] = (int32_t)(k0 + i);
      l_off[lf] = lc;
      ++lf;
    }
    lc += c[i];
  }
  if (wave == 0) {
    const int64_t base = (tile == 0 && lane == 0) ? *s.cursor : 0;
    const int64_t bc = lookback(s.state_c, tile, acc_c, __shfl(base, 0), s.epoch);
    if (lane == 0) s_base_c = bc;
  } else if (wave == 1) {
    const int64_t bf = lookback(s.state_f, tile, acc_f, 0, s.epoch);
    if (lane == 0) s_base_f = bf;
  }
  __syncthreads();
  const int64_t bc = s_base_c, bf = s_base_f;
  if (tid == 0 && tile == s.num_tiles - 1) {
    *s.cursor = bc + acc_c;
    *s.list_len = bf + acc_f;
    atomicAdd(s.event_particles, (unsigned long long)(bf + acc_f));
  }
  for (int j = tid; j < acc_f; j += kScanThreads) {
    s.list[bf + j] = l_idx[j];
    s.offsets[bf + j] = bc + l_off[j];
  }
  if (s.offsets_k) {  // every particle's first-child offset (read by the replay)
    int64_t o = bc + pre_c + ic - my_c;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (k0 + i < s.n) s.offsets_k[k0 + i] = o;
      o += c[i];
    }
  }
}

// ------------------------------------------------------------------ write kernels
// Child records are staged per lane in LDS, kLinePieces 16-byte pieces (a
// 64-byte half line of the append buffer) at a time, by the rule of
// line_rule.h, and each half line is written out by kLinePieces lanes.
template <typename T>
using ChildLine = LineState<uint4, (int)(sizeof(Rec<T>) / 16)>;

// kL pieces per line; a lane's slot holds kL + 1 pieces (the spare one puts
// neighbouring slots in different banks)
template <int kL, typename T>
__device__ __forceinline__ void stage_child(uint4* slot, ChildLine<T>& cl, const Rec<T>* base, int64_t o,
                                            const Rec<T>& r) {
  const RecBits<T> b = rec_pack<T>(r);
  line_put<kL>(slot, cl, reinterpret_cast<uint64_t>(base + o) >> 4, b.c);
}

// Writes the line of every lane whose last record reached the end of it
// (running past it or not) or whose parent finished (fin), kL lanes per line.
// Called by the whole wave.
template <int kL, typename T>
__device__ __forceinline__ void line_flush(uint4* wave_slots, uint8_t* owners, ChildLine<T>& cl, bool fin) {
  static_assert(kL == 4 || kL == 8, "half or whole 128-byte lines");
  constexpr uint32_t kPerRound = 64 / kL;
  constexpr int kShift = kL == 8 ? 3 : 2;
  constexpr int kSlot = kL + 1;
  const int lane = lane_id();
  bool ready = line_ready(cl, fin);
  uint64_t rm = __ballot(ready);
  while (rm) {
    const uint32_t r = (uint32_t)__popcll(rm);
    if (ready) owners[mbcnt(rm)] = (uint8_t)lane;
    for (uint32_t g0 = 0; g0 < r; g0 += kPerRound) {
      const uint32_t g = g0 + (uint32_t)(lane >> kShift);
      const int owner = g < r ? (int)owners[g] : lane;
      const uint64_t oln = __shfl(cl.ln, owner);
      const uint32_t om = __shfl(cl.mask, owner);
      const int piece = lane & (kL - 1);
      if (g < r && ((om >> piece) & 1u))
        gptr<uint4>(oln << (kShift + 4))[piece] = wave_slots[owner * kSlot + piece];
    }
    if (ready) ready = line_advance(wave_slots + lane * kSlot, cl, fin);
    rm = __ballot(ready);
  }
}

// The direct write kernel: re-runs every particle with events from the event
// list.  With the event log on it only runs when the log overflowed (the
// replay below does the writes otherwise).
template <typename T, bool kMain, bool kStage>
__global__ void __launch_bounds__(kStage ? kWriteThreads : kStepThreads) k_write_lepton(StepArgs<T> a) {
  constexpr int kThreads = kStage ? kWriteThreads : kStepThreads;
  if (a.log_on) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(&a.stats[kStatLogNeed], a.log_ctl[kLogNeed]);
    if (!a.log_ctl[kLogOverflow]) return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.stats[kStatReruns], 1ull);
  extern __shared__ float lds[];
  __shared__ uint8_t owners[kStage ? kThreads / 64 : 1][64];
  const LdsTables lt = stage_tables<T, false>(a, lds);
  uint4* wave_slots = nullptr;
  if constexpr (kStage) {
    const size_t off = line_stage_offset(sizeof(SrcTable), sizeof(T) == 4, a.tab.rate[0].n,
                                         a.tab.cdf[0].rows32 * a.tab.cdf[0].cols32);
    wave_slots = reinterpret_cast<uint4*>(reinterpret_cast<char*>(lds) + off) + (threadIdx.x & ~63u) * kLineSlot;
  }
  const uint64_t n = (uint64_t)*a.list_len;
  const uint32_t waves = gridDim.x * (kThreads / 64);
  WaveQueue wq;
  wq_init(wq);
  Lane<T> L;
  Outbox<T> O;
  O.what = 0;
  ChildLine<T> cl;
  line_init(cl);
  T q = T(-1);
  int64_t obase = 0;
  bool have = false;
  while (true) {
    const uint64_t e = wq_take(wq, !have, n, a.queue + kQueueWords, waves);
    if (!have && e < n) {
      const int64_t k = a.list[e];
      load_state<T, kMain>(a, lt.src, k, L);
      if (!kMain) load_fields<T>(lt.src, L.root, L.E, L.B);
      obase = a.offsets[e];
      q = a.species + L.part == 0 ? T(-1) : T(1);
      have = true;
    }
    if (!__any(have)) break;  // every lane's last half line went out with its parent's last trip
    bool fin = false;
    if (have) {
      fin = lepton_iter<T, true>(a, lt, L, q, obase, O);
      if (fin) stage_final<T>(a, L, true, false, true, O);
      if constexpr (kStage) {
        if (O.what & kOutChild) {
          stage_child<kLinePieces, T>(wave_slots + lane_id() * kLineSlot, cl, a.out_rec[0], O.at, O.r);
          if (a.positions) {
            T* qp = a.out_pos[0] + 4 * O.at;
            qp[0] = O.x[0];
            qp[1] = O.x[1];
            qp[2] = O.x[2];
            qp[3] = T(0);
          }
          O.what &= ~kOutChild;
        }
      }
      flush<T>(a, lt.src, O);
      if (fin) have = false;
    }
    if constexpr (kStage) line_flush<kLinePieces, T>(wave_slots, owners[threadIdx.x >> 6], cl, fin);
  }
}

// advance_lepton with push and positions fixed at compile time (the replay is
// instantiated for each combination, so that unused state takes no registers);
// the same operations in the same order
template <typename T, bool kPush, bool kPos>
__device__ __forceinline__ void advance_lepton_ct(Lane<T>& L, T q, T h) {
  if constexpr (kPush) boris<T>(L.p, q, L.E, L.B, h);
  if constexpr (kPos) {
    const T gi = T(1) / sqrt(T(1) + L.p[0] * L.p[0] + L.p[1] * L.p[1] + L.p[2] * L.p[2]);
    L.x[0] += L.p[0] * gi * h;
    L.x[1] += L.p[1] * gi * h;
    L.x[2] += L.p[2] * gi * h;
  }
}

// One event replayed from the log: the arithmetic of lepton_iter's event
// branch with z and h taken from the log (the event's draws come from the
// same Philox counters), so the child record and the particle's state come
// out bit for bit the same.
template <typename T, bool kPush, bool kPos>
__device__ __forceinline__ void replay_event(const StepArgs<T>& a, Lane<T>& L, T q, T z, T h, int64_t obase,
                                             Outbox<T>& O) {
  advance_lepton_ct<T, kPush, kPos>(L, q, h);
  L.t += h;
  T d, omd;
  sigmoid_of<T>(z, d, omd);
  const int64_t o = obase + L.j;
  if (o < a.out_cap) {  // the photon: k = delta p, born here
    const uint32_t u = draw(a.seed, L.id, a.step, (uint32_t)L.j).z;
    const uint4 v = draw(a.seed, L.id, a.step, (uint32_t)L.j | 0x80000000u);
    O.r.px = d * L.p[0];
    O.r.py = d * L.p[1];
    O.r.pz = d * L.p[2];
    O.r.tb = L.t;
    O.r.tau = exp_depth_t<T>(u);
    O.r.id = (uint64_t)v.x | ((uint64_t)v.y << 32);
    O.r.w = L.w;
    O.r.root = L.root;
    O.r.nev = 0;
    O.r.alive = 1u;
    if constexpr (kPos) {
      O.x[0] = L.x[0];
      O.x[1] = L.x[1];
      O.x[2] = L.x[2];
    }
    O.at = o;
    O.what = kOutChild;
  }
  L.p[0] *= omd;
  L.p[1] *= omd;
  L.p[2] *= omd;
  L.changed = true;
  ++L.j;
}

// The lepton write pass from the count pass's event log.  It runs the count
// launch's grid, and wave w reads the records of count wave w: its lanes hold
// the same particles on the same trips.  A new lane loads its particle, an
// event lane replays the event and writes the child at the particle's first
// child offset plus the event index, and a lane whose particle finished moves
// it to the end of the step and stores its final state with the logged
// optical depth.  No tables are needed, so LDS holds only the source table
// and (FP32) a whole 128-byte line per lane for the child records, written
// out by eight lanes per line.
constexpr int kReplayLine = 8;
template <typename T, bool kMain, bool kStage, bool kPush, bool kPos>
__global__ void __launch_bounds__(kStepThreads, sizeof(T) == 4 ? kStepWavesPerSimd : 1) k_replay_lepton(StepArgs<T> a) {
  if (!a.log_on || a.log_ctl[kLogOverflow]) return;  // the direct write kernel does the writes
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.stats[kStatReplays], 1ull);
  extern __shared__ float lds[];
  __shared__ uint8_t owners[kStage ? kStepThreads / 64 : 1][64];
  SrcTable* src = reinterpret_cast<SrcTable*>(lds);
  stage_sources<T>(a, src);
  __syncthreads();
  constexpr int kSlot = kReplayLine + 1;
  uint4* wave_slots = nullptr;
  if constexpr (kStage)
    wave_slots = reinterpret_cast<uint4*>(reinterpret_cast<char*>(lds) + sizeof(SrcTable)) +
                 (threadIdx.x & ~63u) * kSlot;
  const uint32_t wave = blockIdx.x * (kStepThreads / 64) + (threadIdx.x >> 6);
  const uint64_t head = a.log_head[wave];
  if (head == 0) return;
  constexpr uint32_t S = log_slot_bytes<T>();
  constexpr uint64_t R = log_record_bytes(S);
  const T dtT = (T)a.dt;
  const int lane = lane_id();
  const uint64_t me = 1ull << lane;
  uint64_t blk = head - 1;
  uint32_t pos = 0;
  // a record (header words m_fresh, m_ev | base, tag, and the lane's slot)
  // and, fetched while the current one is handled, the next
  auto fetch = [&](uint32_t p, uint4& h0, uint4& h1, LogSlot<T>& sl) {
    const char* r = a.log_pool + blk + (uint64_t)p * R;
    h0 = reinterpret_cast<const uint4*>(r)[0];
    h1 = reinterpret_cast<const uint4*>(r)[1];
    sl = *reinterpret_cast<const LogSlot<T>*>(r + kLogHeader + (uint64_t)S * lane);
  };
  uint4 h0, h1;
  LogSlot<T> sl;
  fetch(pos, h0, h1, sl);
  Lane<T> L;
  Outbox<T> O;
  O.what = 0;
  ChildLine<T> cl;
  line_init(cl);
  T q = T(-1);
  int64_t obase = 0;
  bool have = false;
  while (true) {
    const uint64_t m_fresh = join64(h0.x, h0.y), m_ev = join64(h0.z, h0.w);
    const uint64_t tag = join64(h1.z, h1.w);
    if (tag != kLogRecord) {
      if (tag == kLogEnd) break;
      blk = join64(h1.x, h1.y);  // kLogJump: the block the log goes on in
      pos = 0;
      fetch(pos, h0, h1, sl);
      continue;
    }
    // the next record (a record never sits at a block's last position)
    uint4 h0_n, h1_n;
    LogSlot<T> sl_n;
    fetch(pos + 1, h0_n, h1_n, sl_n);
    const bool ev = (m_ev & me) != 0;
    const bool fin = have && !ev;
    if (m_fresh & m_ev & me) {  // a new particle with an event (log_fresh_index)
      const int64_t k = (int64_t)(join64(h1.x, h1.y) + mbcnt(m_fresh));
      load_state<T, kMain, kPush>(a, src, k, L);
      if (!kMain && kPush) load_fields<T>(src, L.root, L.E, L.B);
      if constexpr (!kPos) L.x[0] = L.x[1] = L.x[2] = T(0);
      obase = a.offsets_k[k];
      q = a.species + L.part == 0 ? T(-1) : T(1);
      have = true;
    }
    if (ev) {
      T z, h;
      if constexpr (sizeof(T) == 4) {
        z = __builtin_bit_cast(float, sl.x);
        h = __builtin_bit_cast(float, sl.y);
      } else {
        z = __builtin_bit_cast(double, join64(sl.x, sl.y));
        h = __builtin_bit_cast(double, join64(sl.z, sl.w));
      }
      replay_event<T, kPush, kPos>(a, L, q, z, h, obase, O);
    } else if (fin) {
      const double tf = __builtin_bit_cast(double, join64(sl.x, sl.y));
      if (L.t < dtT) {  // no event before the end of the step (the count pass's last trip)
        advance_lepton_ct<T, kPush, kPos>(L, q, dtT - L.t);
        L.t = dtT;
      }
      L.tau = tf;
      stage_final<T>(a, L, true, false, true, O);
    }
    if constexpr (kStage) {
      if (O.what & kOutChild) {
        stage_child<kReplayLine, T>(wave_slots + lane * kSlot, cl, a.out_rec[0], O.at, O.r);
        if constexpr (kPos) {
          T* qp = a.out_pos[0] + 4 * O.at;
          qp[0] = O.x[0];
          qp[1] = O.x[1];
          qp[2] = O.x[2];
          qp[3] = T(0);
        }
        O.what &= ~kOutChild;
      }
    }
    flush<T>(a, src, O);
    if constexpr (kStage) line_flush<kReplayLine, T>(wave_slots, owners[threadIdx.x >> 6], cl, fin);
    if (fin) have = false;
    h0 = h0_n;
    h1 = h1_n;
    sl = sl_n;
    pos += 1;
  }
}

template <typename T>
__global__ void __launch_bounds__(kStepThreads, sizeof(T) == 4 ? kStepWavesPerSimd : 1) k_write_photon(StepArgs<T> a) {
  extern __shared__ float lds[];
  const LdsTables lt = stage_tables<T, true>(a, lds);
  const int64_t n = *a.list_len;
  for (int64_t e = (int64_t)blockIdx.x * kStepThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kStepThreads) {
    const int64_t k = a.list[e];
    Lane<T> L;
    load_lane<T>(a, lt.src, k, L);
    photon_iter<T, true>(a, lt, L, a.offsets[e]);
    store_final<T>(a, lt.src, L, false, true);  // the photon is removed at its event
  }
}

// ------------------------------------------------------------------ resampling (after the merge)
// Photon energy filter (Sec. 4.2: photons too soft ever to produce a pair
// need not join the ensemble) and global leveling (Sec. 5.1: one threshold
// weight w_th per species; a particle lighter than w_th stays with probability
// w / w_th and then weighs w_th, heavier ones stay as they are).  w_th solves
// sum_i min(1, w_i / w_th) = n_target over the particles that pass the filter;
// the host finds it from the sums below (api.cpp).

// |k|^2 >= e_min^2 in FP64, summed left to right without contraction
template <typename T>
__device__ __forceinline__ bool passes_filter(const SpeciesView<T>& s, int64_t i, bool photon, double e_min2) {
#pragma clang fp contract(off)
  if (!photon || !(e_min2 > 0.0)) return true;
  const double px = s.px[i], py = s.py[i], pz = s.pz[i];
  return px * px + py * py + pz * pz >= e_min2;
}

// One pass of the threshold solve, in two kernels.  k_level_partials: per
// block, over the particles that pass the filter, the weight below wt, the
// total weight, the count at or above wt and the count (a fixed grid and a
// fixed reduction order make the sums reproducible).  k_level_step: one block
// adds the blocks' sums in block order and takes the next step of the solve:
//   first pass (wt = infinity): w_0 = total weight / target when more than
//     `target` particles pass the filter, else done with wt = 0;
//   later passes: w <- S(w) / (target - C(w)), done when that no longer
//     decreases w (or target - C(w) <= 0).
// The state stays on the device and both kernels return at once when the
// solve is done, so a fixed number of passes can be queued without waiting
// for the host; the kernel boundary orders the sums before their total.
template <typename T>
__global__ void __launch_bounds__(kLevelThreads) k_level_partials(SpeciesView<T> s, int64_t n, int32_t photon,
                                                                   double e_min2, int32_t first, const LevelState* ls,
                                                                   double* part) {
  __shared__ double red[4][kLevelThreads];
  if (!first && ls->done) return;
  const double wt = first ? INFINITY : ls->wt;
  double bw = 0.0, aw = 0.0, ca = 0.0, ce = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kLevelThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLevelThreads) {
    if (!passes_filter<T>(s, i, photon != 0, e_min2)) continue;
    const double w = s.w[i];
    ce += 1.0;
    aw += w;
    if (w < wt) bw += w;
    else ca += 1.0;
  }
  red[0][threadIdx.x] = bw;
  red[1][threadIdx.x] = aw;
  red[2][threadIdx.x] = ca;
  red[3][threadIdx.x] = ce;
  __syncthreads();
  for (int h = kLevelThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[(size_t)blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(kLevelThreads) k_level_step(const double* part, int nblocks, int32_t first,
                                                               double target, LevelState* ls) {
  __shared__ double red[4][kLevelThreads];
  if (!first && ls->done) return;
  const double wt = first ? INFINITY : ls->wt;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kLevelThreads)
    for (int q = 0; q < 4; ++q) acc[q] += part[(size_t)b * 4 + q];
  for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int h = kLevelThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double below = red[0][0], total = red[1][0], above = red[2][0], count = red[3][0];
  if (first) {
    ls->eligible = count;
    ls->total = total;
    ls->iterations = 0;
    if (target > 0.0 && count > target) {
      ls->wt = total / target;
      ls->done = 0;
    } else {
      ls->wt = 0.0;
      ls->done = 1;
    }
    return;
  }
  ls->iterations += 1;
  const double room = target - above;
  if (!(room > 0.0)) {
    ls->done = 1;
  } else {
    const double next = below / room;
    if (next < wt)
      ls->wt = next;
    else
      ls->done = 1;
  }
}

// Stable in-place compaction of the survivors (the tile scheme of the photon
// merge): a particle stays if it passes the filter and, when wt > 0, if
// w >= wt or its draw u = (x + 1/2) 2^-32 is below w / wt; a light survivor
// then weighs wt.
template <typename T>
__global__ void __launch_bounds__(kMergeThreads) k_resample(ResampleArgs<T> a) {
  __shared__ int32_t wsum[kMergeThreads / 64];
  __shared__ int64_t s_tile, s_base;
  const int tid = threadIdx.x;
  if (tid == 0) s_tile = (int64_t)atomicAdd(a.ticket, 1ull);
  __syncthreads();
  const int64_t tile = s_tile;
  const SpeciesView<T>& s = a.s;
  T p[kMergeItems][3], x[kMergeItems][3];
  float w[kMergeItems];
  double tau[kMergeItems];
  uint64_t id[kMergeItems];
  uint32_t okmask = 0;
#pragma unroll
  for (int it = 0; it < kMergeItems; ++it) {
    const int64_t g = tile * kMergeTile + (int64_t)it * kMergeThreads + tid;
    bool ok = false;
    if (g < a.n && passes_filter<T>(s, g, a.photon != 0, a.e_min2)) {
      w[it] = s.w[g];
      id[it] = s.id[g];
      ok = true;
      if (a.wt > 0.0 && (double)w[it] < a.wt) {
        const double u = ((double)draw(a.seed, id[it], a.step, kResampleJ).x + 0.5) * 0x1p-32;
        ok = u < (double)w[it] / a.wt;
        w[it] = (float)a.wt;
      }
      if (ok) {
        p[it][0] = s.px[g];
        p[it][1] = s.py[g];
        p[it][2] = s.pz[g];
        if (a.positions) {
          x[it][0] = s.x[g];
          x[it][1] = s.y[g];
          x[it][2] = s.z[g];
        }
        tau[it] = s.tau[g];
      }
    }
    okmask |= (ok ? 1u : 0u) << it;
  }
  // every load of the tile must have returned before its aggregate is
  // published (later tiles write into this tile's range)
#pragma unroll
  for (int it = 0; it < kMergeItems; ++it) {
    if ((okmask >> it) & 1u) {
      asm volatile("" ::"v"(p[it][0]), "v"(p[it][1]), "v"(p[it][2]), "v"(w[it]), "v"(tau[it]), "v"(id[it])
                   : "memory");
      if (a.positions) asm volatile("" ::"v"(x[it][0]), "v"(x[it][1]), "v"(x[it][2]) : "memory");
    }
  }
  int32_t pre[kMergeItems];
  const int lane = lane_id(), wave = tid >> 6;
  int32_t tile_total = 0;
  for (int it = 0; it < kMergeItems; ++it) {
    const uint64_t m = __ballot((okmask >> it) & 1u);
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int32_t before = 0, all = 0;
    for (int wv = 0; wv < kMergeThreads / 64; ++wv) {
      before += wv < wave ? wsum[wv] : 0;
      all += wsum[wv];
    }
    pre[it] = tile_total + before + (int32_t)mbcnt(m);
    tile_total += all;
    __syncthreads();
  }
  if (tid < 64) {
    const int64_t b = lookback(a.state, tile, tile_total, 0, a.epoch);
    if (tid == 0) {
      s_base = b;
      if (tile == a.num_tiles - 1) *a.out_count = b + tile_total;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kMergeItems; ++it) {
    if ((okmask >> it) & 1u) {
      const int64_t o = s_base + pre[it];
      s.px[o] = p[it][0];
      s.py[o] = p[it][1];
      s.pz[o] = p[it][2];
      if (a.positions) {
        s.x[o] = x[it][0];
        s.y[o] = x[it][1];
        s.z[o] = x[it][2];
      }
      s.w[o] = w[it];
      s.tau[o] = tau[it];
      s.id[o] = id[it];
      if (s.alive) s.alive[o] = 1;
    }
  }
}

// ------------------------------------------------------------------ optical depth of new particles
template <typename T>
__global__ void k_init_tau(double* tau, const uint64_t* id, int64_t n, uint64_t seed, uint32_t step) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (tau[i] < 0.0) tau[i] = exp_depth(draw(seed, id[i], step, 0xFFFFFFFFu).x);
}

// ------------------------------------------------------------------ validation kernels
template <typename T>
__global__ void k_eval_rate(TableView tab, int process, const T* chi, const T* energy, T* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if constexpr (sizeof(T) == 4) {
    const RateView& r = tab.rate[process];
    out[i] = process == 0 ? rate_rad32(r.herm, r.n, r.hs_lo, r.inv_h, chi[i], energy[i])
                          : rate_pair32(r.herm, r.n, r.hs_lo, r.inv_h, chi[i], energy[i]);
  } else {
    out[i] = process == 0 ? rate_rad64(tab.rate[0], chi[i], energy[i]) : rate_pair64(tab.rate[1], chi[i], energy[i]);
  }
}

template <typename T>
__global__ void k_eval_particles(TableView tab, int species, const T* px, const T* py, const T* pz, FieldView<T> f,
                                 int64_t n, T* chi_out, T* w_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T p[3] = {px[i], py[i], pz[i]};
  const int64_t o = f.stride ? i : 0;
  const T E[3] = {f.ex[o], f.ey[o], f.ez[o]}, B[3] = {f.bx[o], f.by[o], f.bz[o]};
  T e, chi;
  bool can_pair = false;
  if (species == 2) {
    can_pair = photon_chi<T>(p, E, B, e, chi);
  } else {
    e = sqrt(T(1) + p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    chi = chi_of<T>(p, e, E, B);
  }
  T w;
  if constexpr (sizeof(T) == 4) {
    const RateView& r = tab.rate[species == 2 ? 1 : 0];
    w = species == 2 ? (can_pair ? rate_pair32(r.herm, r.n, r.hs_lo, r.inv_h, chi, e) : 0.f)
                     : rate_rad32(r.herm, r.n, r.hs_lo, r.inv_h, chi, e);
  } else {
    w = species == 2 ? (can_pair ? rate_pair64(tab.rate[1], chi, e) : 0.0) : rate_rad64(tab.rate[0], chi, e);
  }
  if (chi_out) chi_out[i] = chi;
  if (w_out) w_out[i] = w;
}

template <typename T>
__device__ __forceinline__ T sample_one(const TableView& tab, int process, T chi, uint32_t k) {
  T v, omv;
  if constexpr (sizeof(T) == 4) {
    if (process == 0) sample_rad32(tab.cdf[0].f32, tab.cdf[0], chi, k, v, omv);
    else sample_pair32(tab.cdf[1].f32, tab.cdf[1], chi, k, v, omv);
  } else {
    if (process == 0) sample_rad64(tab.cdf[0], chi, k, v, omv);
    else sample_pair64(tab.cdf[1], chi, k, v, omv);
  }
  return v;
}

template <typename T>
__global__ void k_sample(TableView tab, int process, const T* chi, const uint32_t* k, T* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = sample_one<T>(tab, process, chi[i], k[i]);
}

// FP32 with 16-byte-aligned columns: four samples per thread, chi, the
// uniforms and the results moved with 16-byte accesses (the last, partial
// group one sample at a time).  The sampler is bound by its arithmetic (two
// logarithms, an exponential and a 4 x 4 interpolation per sample, against
// 12 bytes of memory traffic); four independent samples per thread give the
// scheduler more to overlap with the table loads.
__global__ void __launch_bounds__(256) k_sample4(TableView tab, int process, const float* chi, const uint32_t* k,
                                                 float* out, int64_t n) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= n) return;
  if (i0 + 4 > n) {
    for (int64_t i = i0; i < n; ++i) out[i] = sample_one<float>(tab, process, chi[i], k[i]);
    return;
  }
  const float4 x = *reinterpret_cast<const float4*>(chi + i0);
  const uint4 u = *reinterpret_cast<const uint4*>(k + i0);
  float4 v;
  v.x = sample_one<float>(tab, process, x.x, u.x);
  v.y = sample_one<float>(tab, process, x.y, u.y);
  v.z = sample_one<float>(tab, process, x.z, u.z);
  v.w = sample_one<float>(tab, process, x.w, u.w);
  *reinterpret_cast<float4*>(out + i0) = v;
}

// ------------------------------------------------------------------ merge
// Stable compaction of photons (alive != 0) over the virtual sequence
// main[0, n_main) ++ app[0, n_app) into main, kMergeItems per thread.  Each
// tile holds all its surviving fields in registers before it publishes its
// aggregate, so writes of later tiles (destination <= source within main)
// never overwrite an element that is still to be read.
template <typename T>
__global__ void __launch_bounds__(kMergeThreads) k_merge_photons(MergeArgs<T> a) {
  __shared__ int32_t wsum[kMergeThreads / 64];
  __shared__ int64_t s_tile, s_base;
  const int tid = threadIdx.x;
  if (tid == 0) s_tile = (int64_t)atomicAdd(a.ticket, 1ull);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t ntot = a.n_main + a.n_app;
  T p[kMergeItems][3], x[kMergeItems][3];
  float w[kMergeItems];
  double tau[kMergeItems];
  uint64_t id[kMergeItems];
  uint32_t okmask = 0;
  // item i of this thread: tile * kMergeTile + i * kMergeThreads + tid (coalesced per item)
#pragma unroll
  for (int it = 0; it < kMergeItems; ++it) {
    const int64_t g = tile * kMergeTile + (int64_t)it * kMergeThreads + tid;
    bool ok = false;
    if (g < ntot) {
      if (g < a.n_main) {
        const SpeciesView<T>& s = a.main;
        ok = s.alive[g] != 0;
        if (ok) {
          p[it][0] = s.px[g];
          p[it][1] = s.py[g];
          p[it][2] = s.pz[g];
          if (a.positions) {
            x[it][0] = s.x[g];
            x[it][1] = s.y[g];
            x[it][2] = s.z[g];
          }
          w[it] = s.w[g];
          tau[it] = s.tau[g];
          id[it] = s.id[g];
        }
      } else {
        const int64_t i = g - a.n_main;
        Rec<T> r;
        rec_load<T>(a.app, i, r);
        ok = r.alive != 0;
        if (ok) {
          p[it][0] = r.px;
          p[it][1] = r.py;
          p[it][2] = r.pz;
          if (a.positions) {
            x[it][0] = a.app_pos[4 * i];
            x[it][1] = a.app_pos[4 * i + 1];
            x[it][2] = a.app_pos[4 * i + 2];
          }
          w[it] = r.w;
          tau[it] = r.tau;
          id[it] = r.id;
        }
      }
    }
    okmask |= (ok ? 1u : 0u) << it;
  }
  // The tile's loads must have returned before its aggregate becomes visible
  // (later tiles write into this tile's source range).  Consuming every loaded
  // register in an empty asm makes the compiler wait for the loads here; the
  // block barrier below then orders all waves before the publish.
#pragma unroll
  for (int it = 0; it < kMergeItems; ++it) {
    if ((okmask >> it) & 1u) {
      asm volatile("" ::"v"(p[it][0]), "v"(p[it][1]), "v"(p[it][2]), "v"(w[it]), "v"(tau[it]), "v"(id[it])
                   : "memory");
      if (a.positions) asm volatile("" ::"v"(x[it][0]), "v"(x[it][1]), "v"(x[it][2]) : "memory");
    }
  }
  // order within the tile: item-major, then thread (matches g)
  int32_t pre[kMergeItems];
  const int lane = lane_id(), wave = tid >> 6;
  int32_t tile_total = 0;
  for (int it = 0; it < kMergeItems; ++it) {
    const uint64_t m = __ballot((okmask >> it) & 1u);
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int32_t before = 0, all = 0;
    for (int wv = 0; wv < kMergeThreads / 64; ++wv) {
      before += wv < wave ? wsum[wv] : 0;
      all += wsum[wv];
    }
    pre[it] = tile_total + before + (int32_t)mbcnt(m);
    tile_total += all;
    __syncthreads();
  }
  if (tid < 64) {
    const int64_t b = lookback(a.state, tile, tile_total, 0, a.epoch);
    if (tid == 0) {
      s_base = b;
      if (tile == a.num_tiles - 1) *a.out_count = b + tile_total;
    }
  }
  __syncthreads();
  const SpeciesView<T>& d = a.main;
#pragma unroll
  for (int it = 0; it < kMergeItems; ++it) {
    if ((okmask >> it) & 1u) {
      const int64_t o = s_base + pre[it];
      d.px[o] = p[it][0];
      d.py[o] = p[it][1];
      d.pz[o] = p[it][2];
      if (a.positions) {
        d.x[o] = x[it][0];
        d.y[o] = x[it][1];
        d.z[o] = x[it][2];
      }
      d.w[o] = w[it];
      d.tau[o] = tau[it];
      d.id[o] = id[it];
      d.alive[o] = 1;
    }
  }
}

__global__ void k_count_alive(const uint8_t* a, int64_t n, unsigned long long* out) {
  int64_t c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c += a[i] != 0;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if (lane_id() == 0 && c) atomicAdd(out, (unsigned long long)c);
}

template <typename T>
__global__ void k_count_alive_rec(const Rec<T>* rec, int64_t n, unsigned long long* out) {
  int64_t c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c += rec[i].alive != 0;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if (lane_id() == 0 && c) atomicAdd(out, (unsigned long long)c);
}

// Appends n records after position `at` of a species' arrays (leptons: all
// survive, so this is a plain conversion of the records).
template <typename T>
__global__ void k_append_records(SpeciesView<T> d, int64_t at, const Rec<T>* rec, const T* pos, int64_t n,
                                 int positions) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    Rec<T> r;
    rec_load<T>(rec, i, r);
    const int64_t o = at + i;
    d.px[o] = r.px;
    d.py[o] = r.py;
    d.pz[o] = r.pz;
    d.w[o] = r.w;
    d.tau[o] = r.tau;
    d.id[o] = r.id;
    if (positions) {
      d.x[o] = pos[4 * i];
      d.y[o] = pos[4 * i + 1];
      d.z[o] = pos[4 * i + 2];
    }
  }
}

// ------------------------------------------------------------------ explicit instantiations via launchers
template <typename K, typename A>
hipError_t launch_step_kernel(K kernel, const A& a, int grid, size_t lds, hipStream_t st, int threads = kStepThreads) {
  if (lds > 65536) {  // raise the kernel's dynamic LDS limit once per size (a host call per launch otherwise)
    static std::mutex mu;
    static std::unordered_map<const void*, size_t> set;  // per kernel: the largest limit set so far
    const void* f = reinterpret_cast<const void*>(kernel);
    std::lock_guard<std::mutex> lk(mu);
    size_t& have = set[f];
    if (lds > have) {
      const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      have = lds;
    }
  }
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), lds, st, a);
  return hipGetLastError();
}
template <typename T, bool kPhoton>
hipError_t launch_count(const StepArgs<T>& a, int grid, size_t lds, hipStream_t st) {
  if (kPhoton) return launch_step_kernel(&k_count_photon<T>, a, grid, lds, st);
  if (a.log_on) {
    if (a.from_main) return launch_step_kernel(&k_count_lepton<T, true, true>, a, grid, lds, st);
    return launch_step_kernel(&k_count_lepton<T, false, true>, a, grid, lds, st);
  }
  if (a.from_main) return launch_step_kernel(&k_count_lepton<T, true, false>, a, grid, lds, st);
  return launch_step_kernel(&k_count_lepton<T, false, false>, a, grid, lds, st);
}
template <typename T, bool kPhoton>
hipError_t launch_write(const StepArgs<T>& a, int grid, size_t lds, hipStream_t st, bool stage) {
  if (kPhoton) return launch_step_kernel(&k_write_photon<T>, a, grid, lds, st);
  if constexpr (sizeof(T) == 4) {  // FP64 keeps its tables in HBM and its registers do not fit 1024 threads
    if (stage) {
      if (a.from_main) return launch_step_kernel(&k_write_lepton<T, true, true>, a, grid, lds, st, kWriteThreads);
      return launch_step_kernel(&k_write_lepton<T, false, true>, a, grid, lds, st, kWriteThreads);
    }
  }
  if (a.from_main) return launch_step_kernel(&k_write_lepton<T, true, false>, a, grid, lds, st);
  return launch_step_kernel(&k_write_lepton<T, false, false>, a, grid, lds, st);
}
// The replay runs the count launch's grid (512-thread blocks); FP32 stages its
// child records in LDS half lines.
template <typename T, bool kMain>
hipError_t launch_replay_main(const StepArgs<T>& a, int grid, hipStream_t st) {
  constexpr bool kStage = sizeof(T) == 4;
  const size_t lds = sizeof(SrcTable) + (kStage ? (size_t)kStepThreads * (kReplayLine + 1) * 16 : 0);
  if (a.push) {
    if (a.positions) return launch_step_kernel(&k_replay_lepton<T, kMain, kStage, true, true>, a, grid, lds, st);
    return launch_step_kernel(&k_replay_lepton<T, kMain, kStage, true, false>, a, grid, lds, st);
  }
  if (a.positions) return launch_step_kernel(&k_replay_lepton<T, kMain, kStage, false, true>, a, grid, lds, st);
  return launch_step_kernel(&k_replay_lepton<T, kMain, kStage, false, false>, a, grid, lds, st);
}
template <typename T>
hipError_t launch_replay(const StepArgs<T>& a, int grid, hipStream_t st) {
  return a.from_main ? launch_replay_main<T, true>(a, grid, st) : launch_replay_main<T, false>(a, grid, st);
}
template hipError_t launch_replay<float>(const StepArgs<float>&, int, hipStream_t);
template hipError_t launch_replay<double>(const StepArgs<double>&, int, hipStream_t);

template <typename T>
hipError_t launch_count_photon_merged(const StepArgs<T>& a, int grid, size_t lds, hipStream_t st) {
  return launch_step_kernel(&k_count_photon_merged<T>, a, grid, lds, st);
}
hipError_t launch_scan(const ScanArgs& s, hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3((unsigned)s.num_tiles), dim3(kScanThreads), 0, st, s);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_level_pass(const SpeciesView<T>& s, int64_t n, int photon, double e_min2, int64_t target, int first,
                             double* part, LevelState* ls, hipStream_t st) {
  hipLaunchKernelGGL((k_level_partials<T>), dim3(kLevelBlocks), dim3(kLevelThreads), 0, st, s, n, photon, e_min2,
                     first, ls, part);
  hipLaunchKernelGGL(k_level_step, dim3(1), dim3(kLevelThreads), 0, st, part, kLevelBlocks, first, (double)target, ls);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_resample(const ResampleArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_resample<T>), dim3((unsigned)a.num_tiles), dim3(kMergeThreads), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_merge_photons(const MergeArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_merge_photons<T>), dim3((unsigned)a.num_tiles), dim3(kMergeThreads), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_count_alive(const uint8_t* alive, int64_t n, unsigned long long* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int grid = (int)((n + 255) / 256);
  grid = grid > 4096 ? 4096 : grid;
  hipLaunchKernelGGL(k_count_alive, dim3(grid), dim3(256), 0, st, alive, n, out);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_count_alive_rec(const Rec<T>* rec, int64_t n, unsigned long long* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int grid = (int)((n + 255) / 256);
  grid = grid > 4096 ? 4096 : grid;
  hipLaunchKernelGGL(k_count_alive_rec<T>, dim3(grid), dim3(256), 0, st, rec, n, out);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_append_records(const SpeciesView<T>& dst, int64_t at, const Rec<T>* rec, const T* pos, int64_t n,
                                 int positions, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int grid = (int)((n + 255) / 256);
  grid = grid > 8192 ? 8192 : grid;
  hipLaunchKernelGGL(k_append_records<T>, dim3(grid), dim3(256), 0, st, dst, at, rec, pos, n, positions);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_init_tau(double* tau, const uint64_t* id, int64_t n, uint64_t seed, uint32_t step, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_tau<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tau, id, n, seed, step);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_eval_rate(const TableView& tab, int process, const T* chi, const T* e, T* out, int64_t n,
                            hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_eval_rate<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tab, process, chi, e, out,
                     n);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_eval_particles(const TableView& tab, int species, const T* px, const T* py, const T* pz,
                                 const FieldView<T>& f, int64_t n, T* chi, T* w, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_eval_particles<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tab, species, px, py,
                     pz, f, n, chi, w);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_sample(const TableView& tab, int process, const T* chi, const uint32_t* k, T* out, int64_t n,
                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    if ((((uintptr_t)chi | (uintptr_t)k | (uintptr_t)out) & 15u) == 0) {
      const int64_t nq = (n + 3) / 4;
      hipLaunchKernelGGL(k_sample4, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, tab, process, chi, k, out,
                         n);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL(k_sample<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tab, process, chi, k, out, n);
  return hipGetLastError();
}

template hipError_t launch_count<float, false>(const StepArgs<float>&, int, size_t, hipStream_t);
template hipError_t launch_count<float, true>(const StepArgs<float>&, int, size_t, hipStream_t);
template hipError_t launch_count<double, false>(const StepArgs<double>&, int, size_t, hipStream_t);
template hipError_t launch_count<double, true>(const StepArgs<double>&, int, size_t, hipStream_t);
template hipError_t launch_write<float, false>(const StepArgs<float>&, int, size_t, hipStream_t, bool);
template hipError_t launch_write<float, true>(const StepArgs<float>&, int, size_t, hipStream_t, bool);
template hipError_t launch_write<double, false>(const StepArgs<double>&, int, size_t, hipStream_t, bool);
template hipError_t launch_write<double, true>(const StepArgs<double>&, int, size_t, hipStream_t, bool);
template hipError_t launch_merge_photons<float>(const MergeArgs<float>&, hipStream_t);
template hipError_t launch_level_pass<float>(const SpeciesView<float>&, int64_t, int, double, int64_t, int, double*,
                                                LevelState*, hipStream_t);
template hipError_t launch_level_pass<double>(const SpeciesView<double>&, int64_t, int, double, int64_t, int,
                                                 double*, LevelState*, hipStream_t);
template hipError_t launch_count_photon_merged<float>(const StepArgs<float>&, int, size_t, hipStream_t);
template hipError_t launch_count_photon_merged<double>(const StepArgs<double>&, int, size_t, hipStream_t);
template hipError_t launch_resample<float>(const ResampleArgs<float>&, hipStream_t);
template hipError_t launch_resample<double>(const ResampleArgs<double>&, hipStream_t);
template hipError_t launch_merge_photons<double>(const MergeArgs<double>&, hipStream_t);
template hipError_t launch_init_tau<float>(double*, const uint64_t*, int64_t, uint64_t, uint32_t, hipStream_t);
template hipError_t launch_count_alive_rec<float>(const Rec<float>*, int64_t, unsigned long long*, hipStream_t);
template hipError_t launch_count_alive_rec<double>(const Rec<double>*, int64_t, unsigned long long*, hipStream_t);
template hipError_t launch_append_records<float>(const SpeciesView<float>&, int64_t, const Rec<float>*, const float*,
                                                 int64_t, int, hipStream_t);
template hipError_t launch_append_records<double>(const SpeciesView<double>&, int64_t, const Rec<double>*,
                                                  const double*, int64_t, int, hipStream_t);
template hipError_t launch_eval_rate<float>(const TableView&, int, const float*, const float*, float*, int64_t,
                                            hipStream_t);
template hipError_t launch_eval_rate<double>(const TableView&, int, const double*, const double*, double*, int64_t,
                                             hipStream_t);
template hipError_t launch_eval_particles<float>(const TableView&, int, const float*, const float*, const float*,
                                                 const FieldView<float>&, int64_t, float*, float*, hipStream_t);
template hipError_t launch_eval_particles<double>(const TableView&, int, const double*, const double*, const double*,
                                                  const FieldView<double>&, int64_t, double*, double*, hipStream_t);
template hipError_t launch_sample<float>(const TableView&, int, const float*, const uint32_t*, float*, int64_t,
                                         hipStream_t);
template hipError_t launch_sample<double>(const TableView&, int, const double*, const uint32_t*, double*, int64_t,
                                          hipStream_t);

}  // namespace sfqed
