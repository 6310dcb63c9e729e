// Host model of the staging of child records in the lepton write kernel.
//
// The kernel's lanes each write the children of one parent (contiguous
// records of the append buffer) through a line buffer, by the rule of
// csrc/line_rule.h: a record's 16-byte pieces are collected in the buffer of
// the destination line they fall in, and the line is written out (only its
// filled pieces) when a record reaches the end of the line or the parent is
// finished.  This program runs that same rule on the host, lane by lane, for
// random parents (start records, child counts, the buffer's phase against
// the lines, capacities that cut a parent's children short) and checks that
// the buffer ends up byte for byte as if every record had been stored
// directly, with nothing written past the capacity.
//
// It also runs the rule that preceded the current one -- write a line out
// only when all its pieces are set, or when the parent is finished -- and
// reports whether the model finds it wrong (it should: a parent whose range
// starts in the middle of a line never fills that line, so its next record is
// staged into the wrong line).
//
// Usage: line_rule_model [trials]   exit 0: current rule exact and the earlier
// rule caught; 1 otherwise.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_2409_17299_amd/csrc/line_rule.h"

namespace {

struct Piece {
  uint32_t x, y, z, w;
};
bool same(const Piece& a, const Piece& b) { return a.x == b.x && a.y == b.y && a.z == b.z && a.w == b.w; }
const Piece kUnset{0xABABABABu, 0xABABABABu, 0xABABABABu, 0xABABABABu};

// the pieces of record r (an arbitrary tag per piece)
Piece tag(int64_t r, int k) { return Piece{(uint32_t)r, (uint32_t)k, 0x5EED0000u ^ (uint32_t)r, 7u * (uint32_t)k + 1u}; }

struct Result {
  int64_t trials = 0, bad_trials = 0, misplaced = 0, past_capacity = 0, invariant = 0;
};

// One lane processes `parents` in order.  mem holds the append buffer of
// `cap` records starting at global piece `base`; returns mismatches.
template <int kP, int kL, bool kEarlierRule>
void run_lane(const std::vector<std::pair<int64_t, int>>& parents, int64_t cap, uint64_t base,
              std::vector<Piece>& mem, Result& res) {
  using namespace sfqed;
  LineState<Piece, kP> cl;
  line_init(cl);
  Piece slot[kL];
  for (int i = 0; i < kL; ++i) slot[i] = kUnset;
  auto write_line = [&]() {
    for (int q = 0; q < kL; ++q) {
      if (!((cl.mask >> q) & 1u)) continue;
      const int64_t g = (int64_t)(cl.ln * kL + q) - (int64_t)base;  // piece index within the buffer
      if (g < 0 || g >= (int64_t)mem.size()) {
        ++res.past_capacity;
        continue;
      }
      if (g >= cap * kP) ++res.past_capacity;
      mem[g] = slot[q];
    }
  };
  auto flush = [&](bool fin) {
    bool ready = kEarlierRule ? (cl.ln != kNoLine && (fin || cl.mask == (1u << kL) - 1u)) : line_ready(cl, fin);
    while (ready) {
      write_line();
      ready = line_advance(slot, cl, fin);
    }
  };
  for (const auto& pr : parents) {
    const int64_t o = pr.first;
    const int m = pr.second;
    for (int j = 0; j < m; ++j) {  // one loop trip per event
      const int64_t r = o + j;
      if (r < cap) {
        Piece b[kP];
        for (int k = 0; k < kP; ++k) b[k] = tag(r, k);
        const uint64_t p0 = base + (uint64_t)r * kP;
        if (cl.ln != kNoLine && p0 / kL != cl.ln) ++res.invariant;
        line_put<kL>(slot, cl, p0, b);
      }
      flush(false);
    }
    flush(true);  // the trip on which the parent reaches the end of the step
  }
}

template <int kP, int kL, bool kEarlierRule>
Result trials(int n, uint64_t seed) {
  std::mt19937_64 rng(seed);
  Result res;
  for (int t = 0; t < n; ++t) {
    // a run of parents with consecutive child ranges (as the scan lays them
    // out), dealt to a few lanes
    const int np = 1 + (int)(rng() % 24);
    std::vector<std::pair<int64_t, int>> all;
    int64_t o = (int64_t)(rng() % 7);
    for (int i = 0; i < np; ++i) {
      const int m = (int)(rng() % 4 == 0 ? rng() % 3 : rng() % 40);  // many parents with 0-2 children
      all.push_back({o, m});
      o += m;
    }
    const int64_t total = o;
    const int64_t cap = rng() % 3 == 0 ? (int64_t)(rng() % (uint64_t)(total + 1)) : total;
    const uint64_t base = 1024 + rng() % (uint64_t)kL;  // the buffer's phase against the lines
    std::vector<Piece> mem((size_t)(total + 2 * kL) * kP, kUnset);
    const int lanes = 1 + (int)(rng() % 4);
    std::vector<std::vector<std::pair<int64_t, int>>> per(lanes);
    for (int i = 0; i < np; ++i) per[rng() % lanes].push_back(all[i]);
    Result one;
    for (int l = 0; l < lanes; ++l) run_lane<kP, kL, kEarlierRule>(per[l], cap, base, mem, one);
    // expected: every parent's record below the capacity in place, nothing
    // else written (the records before the first parent belong to no one)
    const int64_t first = all.front().first;
    for (int64_t r = 0; r < total; ++r)
      for (int k = 0; k < kP; ++k) {
        const Piece want = r >= first && r < cap ? tag(r, k) : kUnset;
        if (!same(mem[(size_t)(r * kP + k)], want)) ++one.misplaced;
      }
    for (size_t g = (size_t)total * kP; g < mem.size(); ++g)
      if (!same(mem[g], kUnset)) ++one.misplaced;
    ++res.trials;
    res.misplaced += one.misplaced;
    res.past_capacity += one.past_capacity;
    res.invariant += one.invariant;
    if (one.misplaced || one.past_capacity || one.invariant) ++res.bad_trials;
  }
  return res;
}

template <int kP, int kL>
bool check(const char* name, int n) {
  const Result now = trials<kP, kL, false>(n, 12345 + kP * 10 + kL);
  const Result old = trials<kP, kL, true>(n, 12345 + kP * 10 + kL);
  std::printf("%s: current rule %lld/%lld trials wrong (%lld pieces misplaced, %lld past capacity, %lld off-line "
              "records); earlier rule %lld/%lld trials wrong\n",
              name, (long long)now.bad_trials, (long long)now.trials, (long long)now.misplaced,
              (long long)now.past_capacity, (long long)now.invariant, (long long)old.bad_trials,
              (long long)old.trials);
  return now.bad_trials == 0 && old.bad_trials > 0;
}

}  // namespace

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 20000;
  bool ok = true;
  ok &= check<3, 4>("48-byte records, 64-byte half lines", n);
  ok &= check<4, 4>("64-byte records, 64-byte half lines", n);
  ok &= check<3, 8>("48-byte records, 128-byte lines", n);
  ok &= check<4, 8>("64-byte records, 128-byte lines", n);
  return ok ? 0 : 1;
}
