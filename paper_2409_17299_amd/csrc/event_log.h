// event_log.h -- the format of the lepton count pass's event log, shared by
// the kernels that write and read it (step.hip) and by a host model of both.
//
// Per wave of the count launch, a sequence of records in blocks of kLogBlock
// bytes.  A record has a fixed size, so that the reader can fetch the next
// record before it has read the current one:
//   header, 32 bytes: m_fresh (64-bit mask of the lanes that took a new
//     particle on this trip, with or without an event), m_ev (lanes with an
//     event), base (the launch index of the particle the lowest fresh lane
//     took) and tag (kLogRecord);
//   64 slots of `slot` bytes, slot l for lane l, written only for lanes with
//     an event (the event's sampled value z and its sub-interval h) or whose
//     particle, which had events, finished on this trip (its final optical
//     depth).
// The wave queue serves a trip's fresh lanes from one contiguous range, in
// lane order, so fresh lane l took particle base + (fresh lanes below l).  A
// fresh lane whose particle has no event at all finishes on that trip and is
// never replayed, but it still takes a particle: it counts in that rank.
// A block holds log_records_per_block records; the last position of a block
// is kept for a marker, a header whose tag is kLogEnd (the wave's log ends)
// or kLogJump (the log goes on in the block at offset `base`).
#pragma once

#include <stdint.h>

#if defined(__HIP__)
#define SFQED_HD __host__ __device__
#else
#define SFQED_HD
#endif

namespace sfqed {

constexpr uint64_t kLogBlock = 128 * 1024;
constexpr uint64_t kLogHeader = 32;
constexpr uint64_t kLogRecord = 0;  // tags
constexpr uint64_t kLogEnd = 1;
constexpr uint64_t kLogJump = 2;

SFQED_HD constexpr uint64_t log_record_bytes(uint32_t slot) { return kLogHeader + 64ull * slot; }
SFQED_HD constexpr uint64_t log_records_per_block(uint32_t slot) { return kLogBlock / log_record_bytes(slot); }

// the launch index of fresh lane `lane` of a record
SFQED_HD inline uint64_t log_fresh_index(uint64_t m_fresh, uint64_t base, int lane) {
  const uint64_t below = lane == 0 ? 0ull : (m_fresh & (~0ull >> (64 - lane)));
#if defined(__HIP_DEVICE_COMPILE__)
  return base + (uint64_t)__popcll(below);
#else
  return base + (uint64_t)__builtin_popcountll(below);
#endif
}

}  // namespace sfqed
