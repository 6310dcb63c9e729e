// line_rule.h -- the per-lane state machine that stages a parent's child
// records in a line buffer before they are written out whole.
//
// A lane writes the children of one parent, which are contiguous records in
// the append buffer.  Instead of storing each record at once (a store
// instruction whose 64 lanes touch 64 different lines), the lane collects the
// record's 16-byte pieces in a buffer covering one aligned line of kL pieces
// of the destination (line index = byte address / (16 kL)), and the line is
// written out when a record reaches its end or the parent is finished.  A
// record of kP <= kL pieces that runs past the end of the line keeps its tail
// pieces aside (ov) until the line has been written; they then start the next
// line.
//
// Invariant: while a line is held, the next record of the parent starts inside
// it.  This holds because a line is written out as soon as a record reaches
// its end (eol) -- not when all kL pieces are set, which a parent whose range
// starts in the middle of a line never achieves for its first line.
//
// These functions hold no memory access of their own: the caller passes the
// lane's slot buffer (LDS in the kernel) and performs the write of a ready
// line, so the same rule runs in the kernel and in a host model of it.
#pragma once

#include <stdint.h>

#if defined(__HIP__)
#define SFQED_HD __host__ __device__
#else
#define SFQED_HD
#endif

namespace sfqed {

constexpr uint64_t kNoLine = ~0ull;

template <typename Piece, int kP>
struct LineState {
  uint64_t ln;    // line held (kNoLine: none)
  uint32_t mask;  // slots of the line that hold data
  int32_t first;  // first piece of the last record kept in ov (kP: none)
  bool eol;       // the last record reached the end of the line
  Piece ov[kP];
};

template <typename Piece, int kP>
SFQED_HD inline void line_init(LineState<Piece, kP>& cl) {
  cl.ln = kNoLine;
  cl.mask = 0;
  cl.first = kP;
  cl.eol = false;
}

// Stages the kP pieces b[] of a record whose first piece is global piece p0.
template <int kL, typename Piece, int kP>
SFQED_HD inline void line_put(Piece* slot, LineState<Piece, kP>& cl, uint64_t p0, const Piece (&b)[kP]) {
  static_assert(kP <= kL && (kL & (kL - 1)) == 0, "a record spans at most two lines");
  const int q0 = (int)(p0 & (uint64_t)(kL - 1));
  if (cl.ln == kNoLine) cl.ln = p0 / (uint64_t)kL;
  cl.first = kP;
  cl.eol = q0 + kP >= kL;
#pragma unroll
  for (int k = 0; k < kP; ++k) {
    if (q0 + k < kL) {
      slot[q0 + k] = b[k];
      cl.mask |= 1u << (q0 + k);
    } else {
      cl.ov[k] = b[k];
      if (cl.first == kP) cl.first = k;
    }
  }
}

// The held line is to be written out now: its last record reached the end of
// the line, or the parent has no more records (fin).
template <typename Piece, int kP>
SFQED_HD inline bool line_ready(const LineState<Piece, kP>& cl, bool fin) {
  return cl.ln != kNoLine && (fin || cl.eol);
}

// After the held line has been written: the tail of the last record, if any,
// starts the next line.  Returns whether that line is to be written at once
// too (only when the parent is finished).
template <typename Piece, int kP>
SFQED_HD inline bool line_advance(Piece* slot, LineState<Piece, kP>& cl, bool fin) {
  cl.mask = 0;
  cl.eol = false;
  if (cl.first < kP) {
    cl.ln += 1;
#pragma unroll
    for (int k = 0; k < kP; ++k)
      if (k >= cl.first) {
        slot[k - cl.first] = cl.ov[k];
        cl.mask |= 1u << (k - cl.first);
      }
    cl.first = kP;
    return fin;
  }
  cl.ln = kNoLine;
  return false;
}

}  // namespace sfqed
