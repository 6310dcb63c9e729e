// event_log.h -- the format of the lepton count pass's event log, shared by
// the kernels that write and read it (step.hip) and by a host model of both.
//
// Per wave of the count launch, a sequence of records in blocks of kLogBlock
// bytes.  A record has a fixed size, so that the reader can fetch the next
// record before it has read the current one:
//   header, 16 bytes: m_new (64-bit mask of the lanes that took a new particle
//     with an event on this trip) and m_ev (lanes with an event);
//   64 slots of `slot` bytes, slot l for lane l, written only for lanes with
//     an event (the event's values and the particle's launch index) or whose
//     particle, which had events, finished on this trip (its final optical
//     depth).
// A block holds log_records_per_block records; the last position of a block
// is kept for a marker.  A new lane always has an event on its first logged
// trip, so m_new is a subset of m_ev in every record.  Markers are the
// headers that break that rule: (~0, 0) ends the wave's log, (~0, 1) moves
// to the block whose offset is the first 8 bytes of slot 0.  (A record may
// have m_new = ~0: every lane took a new particle, and then m_ev = ~0 too.)
#pragma once

#include <stdint.h>

#if defined(__HIP__)
#define SFQED_HD __host__ __device__
#else
#define SFQED_HD
#endif

namespace sfqed {

constexpr uint64_t kLogBlock = 128 * 1024;
constexpr uint64_t kLogMarkNew = ~0ull;
constexpr uint64_t kLogMarkEnd = 0;   // m_ev of the end marker
constexpr uint64_t kLogMarkJump = 1;  // m_ev of the jump marker

SFQED_HD constexpr uint64_t log_record_bytes(uint32_t slot) { return 16ull + 64ull * slot; }
SFQED_HD constexpr uint64_t log_records_per_block(uint32_t slot) { return kLogBlock / log_record_bytes(slot); }

// a marker, not a record: some new lane without an event
SFQED_HD inline bool log_is_marker(uint64_t m_new, uint64_t m_ev) { return (m_new & ~m_ev) != 0; }

}  // namespace sfqed
