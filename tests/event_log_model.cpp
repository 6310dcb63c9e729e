// Host model of the lepton count pass's event log and of its replay.
//
// One wave of 64 lanes runs the count pass's lane discipline: a lane without
// a particle takes the next one from the wave's queue at the start of a trip;
// on a trip a lane's particle either has an event or reaches the end of the
// step (finishes).  The queue hands out particles in chunks of consecutive
// indices; as in the count pass with the log on, one trip serves its lanes
// from one chunk only (lanes left over wait a trip).  After each trip the
// writer appends a record (fixed-size records, format of csrc/event_log.h,
// logic of log_trip / log_close in step.hip); the reader then walks the log
// as k_replay_lepton does, fetching each next record ahead and never outside
// the block, and must hand every particle with events its launch index, its
// events' values in order and its final optical depth, and nothing to
// particles without events.  Particles get random event counts, with runs of
// trips on which every lane takes a new particle and fresh lanes whose
// particle has no event at all (they take an index but are never replayed);
// blocks fill and continue in others (jump markers), and the pool runs out in
// some trials (the writer stops, as the kernel does, and nothing is
// replayed).
//
// Two variants must come out wrong: a reader that ranks a new lane among the
// fresh lanes with an event only (it ignores the fresh lanes whose particle
// had none), and a writer whose queue serves one trip from two chunks (the
// fresh lanes' indices are then not consecutive).
//
// Usage: event_log_model [trials]; exit 0: the reader is exact and both
// variants are caught.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../paper_2409_17299_amd/csrc/event_log.h"

namespace {

using namespace sfqed;
constexpr uint32_t kSlot = 8;  // FP32 slots: z and h, or the final optical depth
constexpr uint64_t kRec = log_record_bytes(kSlot);
constexpr uint32_t kPer = (uint32_t)log_records_per_block(kSlot);

struct Particle {
  std::vector<uint32_t> ev;  // per event: a tag standing for (z, h)
  uint64_t tau_final;        // stands for the final optical depth
};

void put64(std::vector<uint8_t>& pool, uint64_t at, uint64_t v) { std::memcpy(&pool[at], &v, 8); }
uint64_t get64(const std::vector<uint8_t>& pool, uint64_t at) {
  uint64_t v;
  std::memcpy(&v, &pool[at], 8);
  return v;
}

struct Writer {
  std::vector<uint8_t>& pool;
  uint64_t cap, used = 0, blk = 0;
  uint32_t pos = 0;
  bool open = false, dead = false, overflow = false;
  uint64_t head = 0;
  int64_t jumps = 0;
  void header(uint64_t at, uint64_t w0, uint64_t w1, uint64_t w2, uint64_t tag) {
    put64(pool, at, w0);
    put64(pool, at + 8, w1);
    put64(pool, at + 16, w2);
    put64(pool, at + 24, tag);
  }
  void trip(const bool* ev, const bool* fin, const bool* fresh, const uint64_t* k, const uint32_t* val,
            const uint64_t* tau) {
    uint64_t m_part = 0, m_fresh = 0, m_ev = 0;
    for (int l = 0; l < 64; ++l) {
      if (ev[l] || fin[l]) m_part |= 1ull << l;
      if (fresh[l]) m_fresh |= 1ull << l;
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
        header(blk + (uint64_t)pos * kRec, 0, 0, b, kLogJump);
      } else {
        head = b + 1;
      }
      open = true;
      blk = b;
      pos = 0;
    }
    const uint64_t base = m_fresh ? k[__builtin_ctzll(m_fresh)] : 0;
    const uint64_t rec = blk + (uint64_t)pos * kRec;
    header(rec, m_fresh, m_ev, base, kLogRecord);
    for (int l = 0; l < 64; ++l) {
      if (!(ev[l] || fin[l])) continue;
      uint32_t v[2];
      if (ev[l]) {
        v[0] = val[l];
        v[1] = val[l] ^ 0x55555555u;
      } else {
        std::memcpy(v, &tau[l], 8);
      }
      std::memcpy(&pool[rec + kLogHeader + (uint64_t)kSlot * l], v, 8);
    }
    pos += 1;
  }
  void close() {
    if (open && !dead) header(blk + (uint64_t)pos * kRec, 0, 0, 0, kLogEnd);
  }
};

struct Replayed {
  std::vector<std::vector<uint32_t>> ev;
  std::vector<uint64_t> tau;
  std::vector<int> done;
  int64_t bad = 0;  // reads outside the pool, unknown particles, values that do not decode
};

// kRankEventLanes: the reader variant that ranks a new lane among the fresh
// lanes with an event only.  The reader fetches each next record before it
// handles the current one, as the kernel does; that fetch must stay inside
// the block.
template <bool kRankEventLanes>
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
    const uint64_t m_fresh = get64(pool, rec), m_ev = get64(pool, rec + 8);
    const uint64_t base = get64(pool, rec + 16), tag = get64(pool, rec + 24);
    if (tag != kLogRecord) {
      if (tag == kLogEnd) return;
      if (tag != kLogJump) {
        ++r.bad;
        return;
      }
      blk = base;
      pos = 0;
      continue;
    }
    if (pos + 1 >= kPer) {  // the fetch of the next record would leave the block
      ++r.bad;
      return;
    }
    for (int l = 0; l < 64; ++l) {
      uint32_t v[2];
      std::memcpy(v, &pool[rec + kLogHeader + (uint64_t)kSlot * l], 8);
      const bool ev = (m_ev >> l) & 1ull;
      if ((m_fresh & m_ev) >> l & 1ull) {
        const uint64_t k = kRankEventLanes ? log_fresh_index(m_fresh & m_ev, base, l)
                                           : log_fresh_index(m_fresh, base, l);
        if (k >= n) {
          ++r.bad;
          return;
        }
        have[l] = (int64_t)k;
      }
      if (ev) {
        if (have[l] < 0) {
          ++r.bad;
          return;
        }
        if (v[1] != (v[0] ^ 0x55555555u)) ++r.bad;
        r.ev[have[l]].push_back(v[0]);
      } else if (have[l] >= 0) {
        // a lane with a particle and no event in a record: it finished
        std::memcpy(&r.tau[have[l]], v, 8);
        r.done[have[l]] += 1;
        have[l] = -1;
      }
    }
    pos += 1;
  }
  ++r.bad;  // no end marker
}

int64_t g_jumps = 0, g_full_new = 0, g_quiet_fresh = 0;

// One wave over n particles; returns mismatches between the particles and
// what the reader hands back (0 = exact).  cap: pool bytes; kTwoChunks: the
// writer variant whose queue may serve a trip from two chunks.
template <bool kRankEventLanes, bool kTwoChunks>
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
  // the queue: chunks of consecutive indices, from 1 to 300 long, in random
  // order (other waves take the chunks in between)
  std::vector<std::pair<size_t, size_t>> chunks;
  for (size_t at = 0; at < n;) {
    const size_t len = std::min<size_t>(n - at, 1 + rng() % 300);
    chunks.push_back({at, at + len});
    at += len;
  }
  std::shuffle(chunks.begin(), chunks.end(), rng);
  size_t ci = 0, next = 0, end = 0;
  std::vector<uint8_t> pool(cap + 64, 0xCD);
  Writer w{pool, cap};
  int64_t part[64];
  int jdone[64];
  for (int l = 0; l < 64; ++l) part[l] = -1;
  while (true) {
    bool fresh[64] = {}, ev[64] = {}, fin[64] = {};
    uint32_t val[64] = {};
    uint64_t tau[64] = {}, kk[64] = {};
    bool served_one = false;
    for (int l = 0; l < 64; ++l) {  // lanes without a particle take the next ones in lane order
      if (part[l] >= 0) continue;
      if (next == end) {
        if (served_one && !kTwoChunks) break;  // one chunk per trip
        if (ci == chunks.size()) break;
        next = chunks[ci].first;
        end = chunks[ci].second;
        ++ci;
      }
      part[l] = (int64_t)next++;
      jdone[l] = 0;
      fresh[l] = true;
      kk[l] = (uint64_t)part[l];
      served_one = true;
    }
    bool any = false;
    for (int l = 0; l < 64; ++l) any |= part[l] >= 0;
    if (!any) break;
    bool all_new = true;
    for (int l = 0; l < 64; ++l) {
      if (part[l] < 0) {
        all_new = false;
        continue;
      }
      const Particle& p = ps[part[l]];
      if (jdone[l] < (int)p.ev.size()) {
        ev[l] = true;
        val[l] = p.ev[jdone[l]++];
      } else {
        fin[l] = jdone[l] > 0;
        g_quiet_fresh += fresh[l] && jdone[l] == 0;
        tau[l] = p.tau_final;
        part[l] = -2;  // finishes on this trip
      }
      all_new &= fresh[l] && ev[l];
    }
    g_full_new += all_new;
    w.trip(ev, fin, fresh, kk, val, tau);
    for (int l = 0; l < 64; ++l)
      if (part[l] == -2) part[l] = -1;
  }
  w.close();
  g_jumps += w.jumps;
  overflowed = w.overflow;
  if (w.overflow) return 0;  // the direct write kernel runs instead
  Replayed r;
  replay<kRankEventLanes>(pool, cap, w.head, n, r);
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

template <bool kRankEventLanes, bool kTwoChunks>
void run(int trials, int64_t& bad_trials, int64_t& overflow_trials) {
  std::mt19937_64 rng(2024);
  bad_trials = overflow_trials = 0;
  for (int t = 0; t < trials; ++t) {
    const size_t n = 1 + rng() % 3000;
    const uint64_t cap = rng() % 8 == 0 ? kLogBlock * (rng() % 3) : kLogBlock * 64;
    bool ov = false;
    if (one_trial<kRankEventLanes, kTwoChunks>(rng, n, cap, ov)) ++bad_trials;
    overflow_trials += ov;
  }
}

}  // namespace

int main(int argc, char** argv) {
  const int trials = argc > 1 ? std::atoi(argv[1]) : 400;
  int64_t bad, ov, bad_rank, ov2, bad_two, ov3;
  run<false, false>(trials, bad, ov);
  const int64_t jumps = g_jumps, full_new = g_full_new, quiet = g_quiet_fresh;
  run<true, false>(trials, bad_rank, ov2);
  run<false, true>(trials, bad_two, ov3);
  std::printf("reader: %lld/%d trials wrong (%lld with the pool exhausted, nothing replayed; %lld block jumps, "
              "%lld trips with every lane new, %lld fresh lanes without events); ranking event lanes only: "
              "%lld/%d wrong; two chunks per trip: %lld/%d wrong\n",
              (long long)bad, trials, (long long)ov, (long long)jumps, (long long)full_new, (long long)quiet,
              (long long)bad_rank, trials, (long long)bad_two, trials);
  return bad == 0 && bad_rank > 0 && bad_two > 0 && jumps > 0 && full_new > 0 && quiet > 0 ? 0 : 1;
}
