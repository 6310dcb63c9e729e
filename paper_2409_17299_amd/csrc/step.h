// step.h -- kernel argument blocks and launchers of the step (host + device).
#pragma once

#include "common.h"
#include "event_log.h"

namespace sfqed {

// step kernels: 8 waves per block, two blocks per CU (the emission tables take
// ~78 KiB of LDS per block), so four waves per SIMD; the FP32 count kernels
// are held to the register budget of that occupancy (the FP64 ones keep their
// tables in HBM and are limited by registers instead).  The lepton write
// kernel runs one block per CU (see kWriteThreads).
constexpr int kStepThreads = 512;
constexpr int kStepWavesPerSimd = 4;
// photons merged inside the step: photons per thread and per tile of the count pass
constexpr int kMergedItems = 4;
constexpr int kMergedTile = kStepThreads * kMergedItems;
// lepton work queue: counters per launch and kernel (see wq_take)
constexpr int kQueueParts = 8;
constexpr int kQueueStride = 16;  // 64-bit words between counters: one 128-byte line each
constexpr int kQueueWords = kQueueParts * kQueueStride;
constexpr uint64_t kChunkMin = 256, kChunkMax = 8192;
// The lepton write kernel runs one block of kWriteThreads per CU (four waves
// per SIMD, one copy of the LDS tables).  Its child records are staged per
// lane in LDS, kLinePieces 16-byte pieces (a 64-byte half line) at a time, and
// written by kLinePieces lanes per half line: a store instruction then covers
// 16 half lines instead of 64 scattered pieces.  A lane's slot has one spare
// piece so that neighbouring slots start in different banks.
constexpr int kWriteThreads = 1024;
constexpr int kLinePieces = 4;
constexpr int kLineShift = 2;  // log2(kLinePieces)
constexpr int kLineSlot = kLinePieces + 1;
constexpr size_t kLineStageBytes = (size_t)kWriteThreads * kLineSlot * 16;
constexpr size_t kMaxLdsBytes = 163840;  // LDS per work-group on gfx950
// byte offset of the line slots in the write kernel's dynamic LDS: after the
// source table and, for FP32, the staged rate and CDF tables
__host__ __device__ constexpr size_t line_stage_offset(size_t src_bytes, int fp32, int rate_n, int cdf_n) {
  return (src_bytes + (fp32 ? 8 * (size_t)rate_n + 4 * (size_t)cdf_n : 0) + 15) / 16 * 16;
}
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kMergeThreads = 256;
constexpr int kMergeItems = 8;
constexpr int kMergeTile = kMergeThreads * kMergeItems;

// device statistics words
constexpr int kStatMaxEvents = 0;
constexpr int kStatCapped = 1;
constexpr int kStatEventParticles = 2;  // + 0 leptons, + 1 photons
constexpr int kStatBadRoot = 4;         // a record's root named no particle of the ensemble
constexpr int kStatLogNeed = 5;         // largest event log a lepton launch needed (bytes)
constexpr int kStatReplays = 6;         // lepton launches written from the event log
constexpr int kStatReruns = 7;          // lepton launches written by the direct write kernel

// Event log of the lepton count pass, replayed by the write pass
// (k_replay_lepton in step.hip; format in event_log.h).  Each wave of the
// count launch writes its own sequence of trip records into blocks handed out
// from one pool; log_ctl words of the launch: blocks handed out, overflow
// flag, bytes the launch needed.
constexpr int kLogUsed = 0, kLogOverflow = 1, kLogNeed = 2;
// bytes of one lane's slot: an event's z and h in the step's dtype, or a
// finished particle's optical depth (FP64)
template <typename T>
constexpr uint32_t log_slot_bytes() {
  return 2u * (uint32_t)sizeof(T);
}

// A launch covers up to two source ranges ("parts"): electrons and positrons
// go together (part 0 e-, part 1 e+), photons alone (part 0).  Particle k of
// the launch is particle begin[0] + k of part 0 for k < n0, else particle
// begin[1] + k - n0 of part 1, so the append order is that of separate
// launches for the two species, one after the other.
// Per-lane choice of launch constants: the step kernels copy the arrays of
// both source ranges and the fields of the three species into this table in
// LDS when they start (see step.hip); it precedes the tables in the dynamic LDS.
enum SrcWord : int { kPx, kPy, kPz, kX, kY, kZ, kW, kTau, kId, kAlive, kNev, kRec, kPos, kBegin, kSrcWords };
enum FieldWord : int { kEx, kEy, kEz, kBx, kBy, kBz, kStride, kFieldCount, kFieldWords };
struct SrcTable {
  uint64_t part[2][kSrcWords];    // the two source ranges of the launch
  uint64_t field[3][kFieldWords];  // the fields of each species
  uint64_t stats;                  // the launch's statistics words (device address)
  uint64_t pad;                    // to a multiple of 16 bytes
};
static_assert(sizeof(SrcTable) % 16 == 0, "LDS layout");

template <typename T>
struct StepArgs {
  SpeciesView<T> src[2];  // the input ensemble of each part (from_main)
  Rec<T>* src_rec[2];     // or its appended records
  T* src_pos[2];          // their positions (4 per record) or null
  int64_t begin[2];       // first particle of each part in its source
  int32_t species;        // species of part 0 (0 e-, 2 photon); part 1 is species + 1
  int32_t from_main;      // 1: sources are the input ensemble (root = species << 30 | index)
  int64_t n0, n;          // particles of part 0; of the launch
  FieldView<T> f[3];
  Rec<T>* out_rec[2];  // leptons: out[0] photons; photons: out[0] e-, out[1] e+
  T* out_pos[2];
  int64_t out_cap;
  int32_t* counts;     // [n]
  int64_t* offsets;    // [n]
  int32_t* list;       // [n]
  const int64_t* list_len;
  unsigned long long* queue;  // work counters of the count, then the write kernel: 2 x kQueueWords, zero at launch
  unsigned long long* stats;
  double dt;
  uint64_t seed;
  uint32_t step;
  int32_t emission, pair, push, positions, write_nev;
  double gamma_min;
  int64_t max_events;
  TableView tab;
  // photons merged inside the step (k_count_photon_merged): survivors of an
  // appended range go straight into the main photon arrays
  SpeciesView<T> dst;               // the main photons
  int64_t dst_cap;                  // their capacity (nothing is written at or past it)
  int64_t* dst_cursor;              // photons in dst so far: read by the first tile, set by the last
  uint64_t* dst_state;              // look-back words, one per tile of kMergedTile photons
  uint32_t dst_epoch;
  unsigned long long* dst_ticket;   // tile counter, zero at launch
  int64_t* pair_cursor;             // pairs appended so far (the scan's cursor of a photon launch)
  // a merged range sized on the device: photons [n_base, min(*n_dev, n_cap)) of
  // the append buffer (the photon cursor after the round's lepton launch), so
  // that the host need not read the cursor back first; null: n photons
  const int64_t* n_dev;
  int64_t n_base, n_cap;
  int64_t list_cap;                 // entries of list and offsets (events past it are not listed)
  // lepton launches: the count pass's event log, replayed by the write pass
  char* log_pool;                   // log blocks
  uint64_t log_cap;                 // bytes of log_pool (0: the count pass only measures the log)
  uint64_t* log_head;               // per wave of the count launch: 1 + byte offset of its first block, 0 = none
  unsigned long long* log_ctl;      // the launch's log words (kLogUsed, kLogOverflow, kLogNeed), zero at launch
  int32_t log_on;                   // 1: the count pass logs; the replay writes unless the log overflowed
  int64_t* offsets_k;               // first-child offset of every particle of the launch (from the scan)
};

struct ScanArgs {
  const int32_t* counts;
  int64_t n;
  int64_t* offsets;
  int32_t* list;
  int64_t* cursor;    // in: append count before the launch; out: after
  int64_t* list_len;
  uint64_t* state_c;  // look-back words, one per tile
  uint64_t* state_f;
  uint32_t epoch;
  unsigned long long* ticket;  // zero at launch
  int64_t num_tiles;
  unsigned long long* event_particles;  // += number of particles with events
  int64_t* offsets_k;  // or null: the first-child offset of every particle
};

template <typename T>
struct MergeArgs {
  SpeciesView<T> main;
  const Rec<T>* app;
  const T* app_pos;
  int64_t n_main, n_app;
  int32_t positions;
  uint64_t* state;
  uint32_t epoch;
  unsigned long long* ticket;
  int64_t num_tiles;
  int64_t* out_count;
};

// resampling after the merge (see step.hip)
constexpr int kLevelThreads = 256;
constexpr int kLevelBlocks = 1024;      // fixed: the sums do not depend on the size of the launch
constexpr uint32_t kResampleJ = 0xFFFFFFFDu;  // Philox counter word of the thinning draw
constexpr int kLevelDevicePasses = 8;   // threshold passes queued without waiting for the host

// Device state of one species' threshold solve (written by k_level_step, read
// by the next pass and by the host).
struct LevelState {
  double wt;        // current threshold weight (0: no thinning)
  double eligible;  // particles that pass the filter
  double total;     // their total weight
  double pad;
  int32_t done, iterations;
};

template <typename T>
struct ResampleArgs {
  SpeciesView<T> s;
  int64_t n;
  int32_t photon, positions;
  double e_min2;  // squared energy threshold of photons (0: no filter)
  double wt;      // leveling threshold weight (0: no leveling)
  uint64_t seed;
  uint32_t step;
  uint64_t* state;
  uint32_t epoch;
  unsigned long long* ticket;
  int64_t num_tiles;
  int64_t* out_count;
};

template <typename T, bool kPhoton>
hipError_t launch_count(const StepArgs<T>& a, int grid, size_t lds, hipStream_t st);
template <typename T>
hipError_t launch_count_photon_merged(const StepArgs<T>& a, int grid, size_t lds, hipStream_t st);
template <typename T, bool kPhoton>
hipError_t launch_write(const StepArgs<T>& a, int grid, size_t lds, hipStream_t st, bool stage = false);
template <typename T>
hipError_t launch_replay(const StepArgs<T>& a, int grid, hipStream_t st);
hipError_t launch_scan(const ScanArgs& s, hipStream_t st);
template <typename T>
hipError_t launch_merge_photons(const MergeArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_level_pass(const SpeciesView<T>& s, int64_t n, int photon, double e_min2, int64_t target, int first,
                             double* part, LevelState* ls, hipStream_t st);
template <typename T>
hipError_t launch_resample(const ResampleArgs<T>& a, hipStream_t st);
hipError_t launch_count_alive(const uint8_t* alive, int64_t n, unsigned long long* out, hipStream_t st);
template <typename T>
hipError_t launch_count_alive_rec(const Rec<T>* rec, int64_t n, unsigned long long* out, hipStream_t st);
template <typename T>
hipError_t launch_append_records(const SpeciesView<T>& dst, int64_t at, const Rec<T>* rec, const T* pos, int64_t n,
                                 int positions, hipStream_t st);
// particles of [0, n) with a non-finite momentum, position, weight, optical
// depth or field component are added to *bad (validate.hip)
template <typename T>
hipError_t launch_count_nonfinite(const SpeciesView<T>& s, const FieldView<T>& f, int64_t n,
                                  unsigned long long* bad, hipStream_t st);
template <typename T>
hipError_t launch_init_tau(double* tau, const uint64_t* id, int64_t n, uint64_t seed, uint32_t step, hipStream_t st);
template <typename T>
hipError_t launch_eval_rate(const TableView& tab, int process, const T* chi, const T* e, T* out, int64_t n,
                            hipStream_t st);
template <typename T>
hipError_t launch_eval_particles(const TableView& tab, int species, const T* px, const T* py, const T* pz,
                                 const FieldView<T>& f, int64_t n, T* chi, T* w, hipStream_t st);
template <typename T>
hipError_t launch_sample(const TableView& tab, int process, const T* chi, const uint32_t* k, T* out, int64_t n,
                         hipStream_t st);


}  // namespace sfqed
