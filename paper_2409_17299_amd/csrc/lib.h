// lib.h -- host-side internals of libsfqed (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/sfqed.h"
#include "common.h"

#define SFQED_HIP(expr)                                       \
  do {                                                        \
    hipError_t e_ = (expr);                                   \
    if (e_ != hipSuccess) {                                   \
      sfqed::set_error(std::string(#expr) + ": " + hipGetErrorString(e_)); \
      return QED_ERR_HIP;                                     \
    }                                                         \
  } while (0)

namespace sfqed {

void set_error(const std::string& msg);

// Geometry of the table grids (host copy of what TableView points to).
struct TableGeom {
  qed_table_cfg cfg;
  int nseg[2];            // Chebyshev segments per process
  double cheb_s_lo[2];
  int herm_n;             // FP32 Hermite nodes per process
  int rows32[2], cols32[2], rows64[2], cols64[2];
  double s0[2], s1[2];    // ln chi of first and last CDF row
  double x0[2], x1[2];    // logit r of first and last CDF column
};

}  // namespace sfqed

struct qed_tables {
  int device;
  sfqed::TableGeom geom;
  sfqed::TableView view;
  void* mem;         // one device allocation holding every table
  size_t bytes;
  size_t off[8];     // export offsets (see qed_tables_export)
  size_t len[8];
};

namespace sfqed {
qed_status build_tables(const qed_table_cfg& cfg, hipStream_t stream, qed_tables* t);

// Scratch words of one merge, provided by the caller: look-back words (tiles
// of them, stamped with epochs; `epoch` must differ from every epoch the
// words still hold) and three control words, the first and third zero on the
// stream before the merge.
struct MergeScratch {
  uint64_t* state;
  int64_t tiles;
  uint32_t epoch;
  uint64_t* ticket;  // tile counter (zero)
  uint64_t* count;   // photons after the merge (written by the last tile)
  uint64_t* alive;   // survivor count when the capacity is tight (zero)
};
template <typename T>
qed_status merge_on(qed_ensemble* ens, const qed_append* app, hipStream_t st, const MergeScratch& ms);
bool merge_args_ok(const qed_ensemble* ens, const qed_append* app);
}
