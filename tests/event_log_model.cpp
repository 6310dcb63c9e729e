// Host model of the lepton count pass's event log and of its replay.
//
// One wave of 64 lanes runs the count pass's lane discipline: a lane without
// a particle takes the next one from the queue at the start of a trip; on a
// trip a lane's particle either has an event or reaches the end of the step
// (finishes).  After each trip the writer appends a record (fixed-size records,
// format and markers of csrc/event_log.h, logic of log_trip / log_close in
// step.hip); the reader then walks the log as k_replay_lepton does, fetching
// each next record ahead and never outside the block, and must hand every
// particle with events its launch index, its events' values in order and its
// final optical depth, and nothing to particles without events.  Particles
// get random event counts, with runs of trips on which every lane takes a new
// particle with an event (the header m_new = ~0), blocks fill and continue in
// others (jump markers), and the pool runs out in some trials (the writer
// stops, as the kernel does, and nothing is replayed).
//
// The model also runs a reader that takes any header with m_new = ~0 for a
// marker -- the reader that faulted on the GPU when every lane of a trip took
// a new particle -- and must find it wrong.
//
// Usage: event_log_model [trials]; exit 0: the reader is exact and the
// earlier reader is caught.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../paper_2409_17299_amd/csrc/event_log.h"

namespace {

using namespace sfqed;
constexpr uint32_t kSlot = 16;  // FP32 slots: z, h, child optical depth, launch index
constexpr uint64_t kRec = log_record_bytes(kSlot);
constexpr uint32_t kPer = (uint32_t)log_records_per_block(kSlot);

struct Particle {
  std::vector<uint32_t> ev;  // per event: a tag standing for (z, h, child tau)
  uint64_t tau_final;        // stands for the final optical depth
};

struct Writer {
  std::vector<uint8_t>& pool;
  uint64_t cap, used = 0, blk = 0;
  uint32_t pos = 0;
  bool open = false, dead = false, overflow = false;
  uint64_t head = 0;
  int64_t jumps = 0;
  void put16(uint64_t at, uint64_t a, uint64_t b) {
    std::memcpy(&pool[at], &a, 8);
    std::memcpy(&pool[at + 8], &b, 8);
  }
  void trip(const bool* ev, const bool* fin, const bool* fresh, const uint32_t* val, const uint64_t* tau,
            const uint64_t* k) {
    uint64_t m_part = 0, m_new = 0, m_ev = 0;
    for (int l = 0; l < 64; ++l) {
      if (ev[l] || fin[l]) m_part |= 1ull << l;
      if (fresh[l] && ev[l]) m_new |= 1ull << l;
      if (ev[l]) m_ev |= 1ull << l;
    }
    if (!m_part || dead) return;
    if (!open || pos + 1 >= kPer) {
      const uint64_t b = used;
      used += kLogBlock;
      if (b + kLogBlock > cap) {
        overflow = true;
        dead = true;
        return;
      }
      if (open) {
        ++jumps;
        const uint64_t m = blk + (uint64_t)pos * kRec;
        put16(m, kLogMarkNew, kLogMarkJump);
        std::memcpy(&pool[m + 16], &b, 8);
      } else {
        head = b + 1;
      }
      open = true;
      blk = b;
      pos = 0;
    }
    const uint64_t rec = blk + (uint64_t)pos * kRec;
    put16(rec, m_new, m_ev);
    for (int l = 0; l < 64; ++l) {
      if (!(ev[l] || fin[l])) continue;
      uint32_t v[4];
      if (ev[l]) {
        v[0] = val[l];
        v[1] = val[l] ^ 0x55555555u;
        v[2] = val[l] + 7u;
        v[3] = (uint32_t)k[l];
      } else {
        std::memcpy(v, &tau[l], 8);
        v[2] = v[3] = 0;
      }
      std::memcpy(&pool[rec + 16 + (uint64_t)kSlot * l], v, 16);
    }
    pos += 1;
  }
  void close() {
    if (open && !dead) put16(blk + (uint64_t)pos * kRec, kLogMarkNew, kLogMarkEnd);
  }
};

struct Replayed {
  std::vector<std::vector<uint32_t>> ev;
  std::vector<uint64_t> tau;
  std::vector<int> done;
  int64_t bad = 0;  // reads outside the pool, unknown particles, values that do not decode
};

// kEarlierReader: any header with m_new = ~0 is taken for a marker.  The reader
// fetches each next record before it handles the current one, as the kernel
// does; that fetch must stay inside the block.
template <bool kEarlierReader>
void replay(const std::vector<uint8_t>& pool, uint64_t cap, uint64_t head, size_t n, Replayed& r) {
  r.ev.assign(n, {});
  r.tau.assign(n, 0);
  r.done.assign(n, 0);
  if (head == 0) return;
  uint64_t blk = head - 1;
  uint32_t pos = 0;
  int64_t have[64];
  for (int l = 0; l < 64; ++l) have[l] = -1;
  for (int guard = 0; guard < 1 << 24; ++guard) {
    if (pos >= kPer || blk + kLogBlock > cap) {
      ++r.bad;
      return;
    }
    const uint64_t rec = blk + (uint64_t)pos * kRec;
    uint64_t m_new, m_ev;
    std::memcpy(&m_new, &pool[rec], 8);
    std::memcpy(&m_ev, &pool[rec + 8], 8);
    const bool marker = kEarlierReader ? m_new == kLogMarkNew : log_is_marker(m_new, m_ev);
    if (marker) {
      if (m_ev == kLogMarkEnd) return;
      std::memcpy(&blk, &pool[rec + 16], 8);
      pos = 0;
      continue;
    }
    if (pos + 1 >= kPer) {  // the fetch of the next record would leave the block
      ++r.bad;
      return;
    }
    for (int l = 0; l < 64; ++l) {
      uint32_t v[4];
      std::memcpy(v, &pool[rec + 16 + (uint64_t)kSlot * l], 16);
      const bool ev = (m_ev >> l) & 1ull;
      if ((m_new >> l) & 1ull) {
        if (v[3] >= n) {
          ++r.bad;
          return;
        }
        have[l] = (int64_t)v[3];
      }
      if (ev) {
        if (have[l] < 0) {
          ++r.bad;
          return;
        }
        if (v[1] != (v[0] ^ 0x55555555u) || v[2] != v[0] + 7u) ++r.bad;
        r.ev[have[l]].push_back(v[0]);
      } else if (have[l] >= 0) {
        std::memcpy(&r.tau[have[l]], v, 8);
        r.done[have[l]] += 1;
        have[l] = -1;
      }
    }
    pos += 1;
  }
  ++r.bad;  // no end marker
}

// One wave over n particles; returns mismatches between the particles and
// what the reader hands back (0 = exact).  cap: pool bytes.
int64_t g_jumps = 0, g_full_new = 0;

template <bool kEarlierReader>
int64_t one_trial(std::mt19937_64& rng, size_t n, uint64_t cap, bool& overflowed) {
  std::vector<Particle> ps(n);
  const int mode = (int)(rng() % 3);
  for (size_t i = 0; i < n; ++i) {
    int ne;
    if (mode == 0) ne = (int)(rng() % 4 == 0 ? 0 : 1 + rng() % 60);  // many events
    else if (mode == 1) ne = (int)(1 + rng() % 3);                   // few, every particle has one
    else ne = (int)(rng() % 2 ? 0 : rng() % 5);                      // sparse
    for (int j = 0; j < ne; ++j) ps[i].ev.push_back((uint32_t)rng() & 0x0FFFFFFFu);
    ps[i].tau_final = rng();
  }
  std::vector<uint8_t> pool(cap + 64, 0xCD);
  Writer w{pool, cap};
  size_t next = 0;
  int64_t part[64];
  int jdone[64];
  for (int l = 0; l < 64; ++l) part[l] = -1;
  while (true) {
    bool fresh[64] = {}, ev[64] = {}, fin[64] = {};
    uint32_t val[64] = {};
    uint64_t tau[64] = {}, kk[64] = {};
    for (int l = 0; l < 64; ++l)  // lanes without a particle take the next ones in lane order
      if (part[l] < 0 && next < n) {
        part[l] = (int64_t)next++;
        jdone[l] = 0;
        fresh[l] = true;
        kk[l] = (uint64_t)part[l];
      }
    bool any = false;
    for (int l = 0; l < 64; ++l) any |= part[l] >= 0;
    if (!any) break;
    for (int l = 0; l < 64; ++l) {
      if (part[l] < 0) continue;
      const Particle& p = ps[part[l]];
      if (jdone[l] < (int)p.ev.size()) {
        ev[l] = true;
        val[l] = p.ev[jdone[l]++];
        kk[l] = (uint64_t)part[l];
      } else {
        fin[l] = jdone[l] > 0;
        tau[l] = p.tau_final;
        part[l] = -2;  // finishes on this trip
      }
    }
    bool all_new = true;
    for (int l = 0; l < 64; ++l) all_new &= fresh[l] && ev[l];
    g_full_new += all_new;
    w.trip(ev, fin, fresh, val, tau, kk);
    for (int l = 0; l < 64; ++l)
      if (part[l] == -2) part[l] = -1;
  }
  w.close();
  g_jumps += w.jumps;
  overflowed = w.overflow;
  if (w.overflow) return 0;  // the direct write kernel runs instead
  Replayed r;
  replay<kEarlierReader>(pool, cap, w.head, n, r);
  int64_t bad = r.bad;
  for (size_t i = 0; i < n; ++i) {
    const bool has = !ps[i].ev.empty();
    if (has) {
      if (r.ev[i] != ps[i].ev || r.done[i] != 1 || r.tau[i] != ps[i].tau_final) ++bad;
    } else if (!r.ev[i].empty() || r.done[i]) {
      ++bad;
    }
  }
  return bad;
}

template <bool kEarlierReader>
void run(int trials, int64_t& bad_trials, int64_t& overflow_trials) {
  std::mt19937_64 rng(2024);
  bad_trials = overflow_trials = 0;
  for (int t = 0; t < trials; ++t) {
    const size_t n = 1 + rng() % 3000;
    const uint64_t cap = rng() % 8 == 0 ? kLogBlock * (rng() % 3) : kLogBlock * 64;
    bool ov = false;
    if (one_trial<kEarlierReader>(rng, n, cap, ov)) ++bad_trials;
    overflow_trials += ov;
  }
}

}  // namespace

int main(int argc, char** argv) {
  const int trials = argc > 1 ? std::atoi(argv[1]) : 400;
  int64_t bad, ov, bad_old, ov_old;
  run<false>(trials, bad, ov);
  run<true>(trials, bad_old, ov_old);
  std::printf("reader: %lld/%d trials wrong (%lld with the pool exhausted, nothing replayed; %lld block jumps, "
              "%lld trips with every lane new); earlier reader: %lld/%d trials wrong\n",
              (long long)bad, trials, (long long)ov, (long long)g_jumps / 2, (long long)g_full_new / 2,
              (long long)bad_old, trials);
  return bad == 0 && bad_old > 0 && g_jumps > 0 && g_full_new > 0 ? 0 : 1;
}
