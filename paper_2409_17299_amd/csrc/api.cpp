// api.cpp -- C ABI of libsfqed: argument checks, per-device scratch, the
// generation-round driver of Algorithm 2 and the merge.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lib.h"
#include "step.h"

namespace sfqed {

namespace {
thread_local std::string g_error;
}
void set_error(const std::string& msg) { g_error = msg; }

namespace {

constexpr int kSlots = 16384;          // zeroed work counters per step
constexpr int kLaunchWords = 2 * kQueueWords + kQueueStride;  // per launch: two queues, the scan ticket
constexpr int kCtrlWords = kSlots + 64;
constexpr int kCurPhoton = kSlots + 0;  // append count of photons
constexpr int kCurLepton = kSlots + 1;  // append count of electrons (= positrons)
constexpr int kListLen = kSlots + 2;
constexpr int kMergeCount = kSlots + 3;
constexpr int kAliveCount = kSlots + 4;
constexpr int kStats = kSlots + 8;      // 8 words
constexpr int kResampleCount = kSlots + 16;  // 3 words: survivors of each species' compaction
constexpr int kMergedCursor = kSlots + 24;   // photons in the main arrays so far (qed_step_merged)
constexpr int kNonFinite = kSlots + 32;      // 3 words: particles with non-finite values (qed_validate)
constexpr size_t kPinBytes = 256;            // pinned host bytes for read-backs

// Library-owned scratch of one device: per-particle counts, offsets and event
// list of the largest launch so far, look-back words, and a control block.
struct Scratch {
  int device = -1;
  int64_t cap = 0;
  int32_t* counts = nullptr;
  int64_t* offsets = nullptr;
  int32_t* list = nullptr;
  int64_t tiles_cap = 0;
  uint64_t* state_c = nullptr;
  uint64_t* state_f = nullptr;
  uint64_t* ctrl = nullptr;
  uint32_t epoch = 0;
  int num_cu = 0;
  size_t max_lds = 0;
  double* level = nullptr;  // partial sums of the leveling threshold solve
  // Newton passes queued per species in the next leveling solve: the last
  // solve's count plus one (the solve usually needs the same number from one
  // step to the next), at most kLevelDevicePasses
  int level_passes[3] = {kLevelDevicePasses, kLevelDevicePasses, kLevelDevicePasses};
  uint64_t* state_m = nullptr;  // look-back words of the merged photon count pass, with their own epochs
  int64_t tiles_m_cap = 0;
  uint32_t epoch_m = 0;
  // the lepton count pass's event log (replayed by the write pass): a pool
  // that grows to the largest launch's need, and one head word per wave
  int64_t* offsets_k = nullptr;  // first-child offset of every particle of a launch
  char* log_pool = nullptr;
  uint64_t log_cap = 0;
  uint64_t* log_head = nullptr;
  int64_t log_waves = 0;
  // pinned host words for small read-backs (a copy into pageable memory goes
  // through a staging buffer: two copies instead of one)
  int64_t* pin = nullptr;
  std::mutex mu;
};

std::mutex g_scratch_mu;
std::vector<Scratch*> g_scratch;

Scratch* scratch_for_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  for (Scratch* s : g_scratch)
    if (s->device == dev) return s;
  Scratch* s = new Scratch();
  s->device = dev;
  int v = 0;
  (void)hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
  s->num_cu = v > 0 ? v : 1;
  (void)hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  s->max_lds = v > 0 ? (size_t)v : 65536;
  if (hipMalloc(&s->ctrl, sizeof(uint64_t) * kCtrlWords) != hipSuccess) {
    delete s;
    return nullptr;
  }
  if (hipMemset(s->ctrl, 0, sizeof(uint64_t) * kCtrlWords) != hipSuccess) {
    delete s;
    return nullptr;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&s->pin), kPinBytes, hipHostMallocDefault) != hipSuccess) {
    s->pin = nullptr;  // read-backs then go to pageable memory
    (void)hipGetLastError();
  }
  g_scratch.push_back(s);
  return s;
}

// Copies `bytes` from the device to dst once `st` has run up to here, through
// the pinned words when they exist and the copy fits.
qed_status read_back(Scratch* S, void* dst, const void* src, size_t bytes, hipStream_t st) {
  void* h = (S->pin && bytes <= kPinBytes) ? static_cast<void*>(S->pin) : dst;
  SFQED_HIP(hipMemcpyAsync(h, src, bytes, hipMemcpyDeviceToHost, st));
  SFQED_HIP(hipStreamSynchronize(st));
  if (h != dst) std::memcpy(dst, h, bytes);
  return QED_OK;
}

qed_status ensure_scratch(Scratch* s, int64_t n) {
  if (n > s->cap) {
    const int64_t cap = std::max<int64_t>(n, s->cap * 3 / 2);
    if (s->counts) {
      SFQED_HIP(hipDeviceSynchronize());
      (void)hipFree(s->counts);
      (void)hipFree(s->offsets);
      (void)hipFree(s->list);
      (void)hipFree(s->offsets_k);
      s->counts = nullptr;
    }
    SFQED_HIP(hipMalloc(&s->counts, sizeof(int32_t) * cap));
    SFQED_HIP(hipMalloc(&s->offsets, sizeof(int64_t) * cap));
    SFQED_HIP(hipMalloc(&s->list, sizeof(int32_t) * cap));
    SFQED_HIP(hipMalloc(&s->offsets_k, sizeof(int64_t) * cap));
    s->cap = cap;
  }
  const int64_t tiles = (std::max(n, s->cap) + kScanTile - 1) / kScanTile + 1;
  if (tiles > s->tiles_cap) {
    if (s->state_c) {
      SFQED_HIP(hipDeviceSynchronize());
      (void)hipFree(s->state_c);
      (void)hipFree(s->state_f);
    }
    SFQED_HIP(hipMalloc(&s->state_c, sizeof(uint64_t) * tiles));
    SFQED_HIP(hipMalloc(&s->state_f, sizeof(uint64_t) * tiles));
    SFQED_HIP(hipMemset(s->state_c, 0, sizeof(uint64_t) * tiles));
    SFQED_HIP(hipMemset(s->state_f, 0, sizeof(uint64_t) * tiles));
    s->tiles_cap = tiles;
    s->epoch = 0;
  }
  return QED_OK;
}

// A look-back word carries the 24-bit epoch of the launch that wrote it, so a
// launch never reads a word left by an earlier one as its own.  When the
// counter wraps, words written 2^24 - 1 launches earlier would match again:
// they are cleared on the stream, ahead of the launch, before epoch 1 is
// reused.  Returns 0 (never a valid epoch) if the clear cannot be queued.
uint32_t next_epoch(Scratch* s, hipStream_t st) {
  s->epoch = (s->epoch + 1) & 0xFFFFFFu;
  if (s->epoch == 0) {
    s->epoch = 1;
    const size_t bytes = sizeof(uint64_t) * (size_t)s->tiles_cap;
    if (bytes && (hipMemsetAsync(s->state_c, 0, bytes, st) != hipSuccess ||
                  hipMemsetAsync(s->state_f, 0, bytes, st) != hipSuccess))
      return 0;
  }
  return s->epoch;
}

uint32_t next_epoch_m(Scratch* s, hipStream_t st) {
  s->epoch_m = (s->epoch_m + 1) & 0xFFFFFFu;
  if (s->epoch_m == 0) {
    s->epoch_m = 1;
    const size_t bytes = sizeof(uint64_t) * (size_t)s->tiles_m_cap;
    if (bytes && hipMemsetAsync(s->state_m, 0, bytes, st) != hipSuccess) return 0;
  }
  return s->epoch_m;
}

// look-back words for `tiles` tiles of the merged photon count pass
qed_status ensure_merged_state(Scratch* s, int64_t tiles) {
  if (tiles <= s->tiles_m_cap) return QED_OK;
  if (s->state_m) {
    SFQED_HIP(hipDeviceSynchronize());
    (void)hipFree(s->state_m);
    s->state_m = nullptr;
  }
  SFQED_HIP(hipMalloc(&s->state_m, sizeof(uint64_t) * tiles));
  SFQED_HIP(hipMemset(s->state_m, 0, sizeof(uint64_t) * tiles));
  s->tiles_m_cap = tiles;
  s->epoch_m = 0;
  return QED_OK;
}

// look-back words for `tiles` tiles of a merge or resampling compaction
qed_status ensure_merge_tiles(Scratch* s, int64_t tiles) {
  if (tiles <= s->tiles_cap) return QED_OK;
  if (s->state_c) {
    SFQED_HIP(hipDeviceSynchronize());
    (void)hipFree(s->state_c);
    (void)hipFree(s->state_f);
  }
  SFQED_HIP(hipMalloc(&s->state_c, sizeof(uint64_t) * tiles));
  SFQED_HIP(hipMalloc(&s->state_f, sizeof(uint64_t) * tiles));
  SFQED_HIP(hipMemset(s->state_c, 0, sizeof(uint64_t) * tiles));
  SFQED_HIP(hipMemset(s->state_f, 0, sizeof(uint64_t) * tiles));
  s->tiles_cap = tiles;
  s->epoch = 0;
  return QED_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// SFQED_WRITE_REPLAY=0 turns the event log off: the lepton write kernel then
// re-runs every particle with events from the tables (the same results).
bool write_replay_enabled() {
  const char* v = std::getenv("SFQED_WRITE_REPLAY");
  return !(v && v[0] == '0');
}

// Head words for the waves of the largest lepton count launch (two blocks of
// kStepThreads per CU).
qed_status ensure_log_heads(Scratch* s) {
  const int64_t waves = (int64_t)s->num_cu * 2 * (kStepThreads / 64);
  if (s->log_head && s->log_waves >= waves) return QED_OK;
  if (s->log_head) {
    SFQED_HIP(hipDeviceSynchronize());
    (void)hipFree(s->log_head);
    s->log_head = nullptr;
  }
  SFQED_HIP(hipMalloc(&s->log_head, sizeof(uint64_t) * waves));
  s->log_waves = waves;
  return QED_OK;
}

// After a step whose lepton launches needed `need` bytes of event log: grow
// the pool to 5/4 of that (whole MiB) when it is short, as long as that takes
// at most half of the free device memory; otherwise launches that need more
// keep the direct write kernel.  Runs with the stream idle.
void grow_log(Scratch* s, uint64_t need) {
  if (need <= s->log_cap) return;
  const uint64_t want = ((need + need / 4) + (1ull << 20) - 1) & ~((1ull << 20) - 1);
  if (s->log_pool) {
    (void)hipDeviceSynchronize();
    (void)hipFree(s->log_pool);
    s->log_pool = nullptr;
    s->log_cap = 0;
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || want > free_b / 2) return;
  if (hipMalloc(&s->log_pool, want) != hipSuccess) {
    s->log_pool = nullptr;
    (void)hipGetLastError();
    return;
  }
  s->log_cap = want;
}

// SFQED_WRITE_STAGING=0 makes the lepton write kernel store every child record
// directly (512-thread blocks) instead of staging it in LDS, so that the two
// paths can be compared byte for byte; both write the same records.
bool write_staging_enabled() {
  const char* v = std::getenv("SFQED_WRITE_STAGING");
  return !(v && v[0] == '0');
}

template <typename T>
SpeciesView<T> view_of(const qed_species& s) {
  SpeciesView<T> v;
  v.px = static_cast<T*>(s.px);
  v.py = static_cast<T*>(s.py);
  v.pz = static_cast<T*>(s.pz);
  v.x = static_cast<T*>(s.x);
  v.y = static_cast<T*>(s.y);
  v.z = static_cast<T*>(s.z);
  v.w = s.w;
  v.tau = s.tau;
  v.id = s.id;
  v.alive = s.alive;
  v.nev = s.nev;
  return v;
}

template <typename T>
FieldView<T> fields_of(const qed_fields& f, int64_t n) {
  FieldView<T> v;
  v.n = n;
  v.ex = static_cast<const T*>(f.ex);
  v.ey = static_cast<const T*>(f.ey);
  v.ez = static_cast<const T*>(f.ez);
  v.bx = static_cast<const T*>(f.bx);
  v.by = static_cast<const T*>(f.by);
  v.bz = static_cast<const T*>(f.bz);
  v.stride = f.stride;
  return v;
}

bool species_ok(const qed_species& s, bool photon, bool positions) {
  if (s.count < 0 || s.capacity < s.count) return false;
  if (s.capacity == 0) return true;
  if (!s.px || !s.py || !s.pz || !s.w || !s.tau || !s.id) return false;
  if (photon && !s.alive) return false;
  const int nx = (s.x != nullptr) + (s.y != nullptr) + (s.z != nullptr);
  if (nx != 0 && nx != 3) return false;
  if ((nx == 3) != positions) return false;
  if (s.capacity >= (int64_t(1) << 30)) return false;  // root index field
  return true;
}

bool append_ok(const qed_append& a, bool positions) {
  if (a.capacity < 0) return false;
  if (a.capacity == 0) return true;
  if (!a.rec || (reinterpret_cast<uintptr_t>(a.rec) & 15u) != 0) return false;
  if (positions && (!a.pos || (reinterpret_cast<uintptr_t>(a.pos) & 15u) != 0)) return false;
  return true;
}

// n particles read these fields: with stride 1 every array must hold n entries
bool fields_ok(const qed_fields& f, int64_t n) {
  if (n == 0) return true;
  if (!f.ex || !f.ey || !f.ez || !f.bx || !f.by || !f.bz) return false;
  return f.stride == 0 || (f.stride == 1 && f.n >= n);
}
std::string fields_error(int s) {
  return "fields of species " + std::to_string(s) +
         ": a missing array, a stride other than 0 or 1, or fewer entries than particles";
}

// HIP events around kernels, read once the step has finished (no extra waits).
struct EventLog {
  bool on = false;
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t begin() {
    if (!on) return nullptr;
    hipEvent_t e = get();
    if (e && hipEventRecord(e, st) != hipSuccess) return nullptr;
    return e;
  }
  void end(int kind, hipEvent_t a) {
    if (!on || !a) return;
    hipEvent_t b = get();
    if (b && hipEventRecord(b, st) == hipSuccess) marks.push_back({kind, {a, b}});
  }
  // after the stream has been synchronised
  void collect(double* ms) {
    for (auto& m : marks) {
      float v = 0.f;
      if (hipEventElapsedTime(&v, m.second.first, m.second.second) == hipSuccess) ms[m.first] += v;
      pool.push_back(m.second.first);
      pool.push_back(m.second.second);
    }
    marks.clear();
  }
  ~EventLog() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    for (auto& m : marks) {
      (void)hipEventDestroy(m.second.first);
      (void)hipEventDestroy(m.second.second);
    }
  }
};

// One launch (count, scan, write) over particles [begin, begin + n) of one
// store.
template <typename T>
qed_status run_launch(Scratch* S, hipStream_t st, const qed_tables* tab, const qed_step_cfg* cfg,
                      const qed_ensemble* ens, qed_append* app, int species, bool from_main, int64_t begin0,
                      int64_t n0, int64_t begin1, int64_t n1, double dt, uint64_t seed, uint32_t step, int* slot,
                      bool positions, EventLog& log, qed_step_stats* stats, bool merged = false,
                      bool device_n = false) {
  // part 0: species, particles [begin0, begin0 + n0); part 1 (leptons): species + 1, [begin1, begin1 + n1).
  // device_n (appended photons of a merged step): n0 is only a bound, the
  // range ends where the photon cursor stands when the launch runs; its events
  // are listed up to the lepton capacity (more pairs overflow anyway)
  const int64_t n = n0 + n1;
  if (n <= 0) return QED_OK;
  const int64_t list_bound = std::min(app[0].capacity, app[1].capacity);
  qed_status rc = ensure_scratch(S, device_n ? std::max<int64_t>(std::min(n, list_bound), 1) : n);
  if (rc != QED_OK) return rc;
  if (*slot + kLaunchWords > kSlots) {
    SFQED_HIP(hipMemsetAsync(S->ctrl, 0, sizeof(uint64_t) * kSlots, st));
    *slot = 0;
  }
  const bool photon = species == 2;
  StepArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  const int parts = n1 > 0 ? 2 : 1;
  for (int q = 0; q < parts; ++q) {
    if (from_main) {
      a.src[q] = view_of<T>(ens->s[species + q]);
    } else {
      a.src_rec[q] = static_cast<Rec<T>*>(app[species + q].rec);
      a.src_pos[q] = static_cast<T*>(app[species + q].pos);
    }
  }
  a.begin[0] = begin0;
  a.begin[1] = begin1;
  a.species = species;
  a.from_main = from_main ? 1 : 0;
  a.n0 = device_n ? INT64_MAX : n0;
  a.n = n;
  a.n_dev = device_n ? reinterpret_cast<const int64_t*>(S->ctrl + kCurPhoton) : nullptr;
  a.n_base = begin0;
  a.n_cap = app[2].capacity;
  a.list_cap = S->cap;
  for (int k = 0; k < 3; ++k) a.f[k] = fields_of<T>(ens->f[k], ens->s[k].count);
  int64_t* cursor;
  if (photon) {
    a.out_rec[0] = static_cast<Rec<T>*>(app[0].rec);
    a.out_rec[1] = static_cast<Rec<T>*>(app[1].rec);
    a.out_pos[0] = static_cast<T*>(app[0].pos);
    a.out_pos[1] = static_cast<T*>(app[1].pos);
    a.out_cap = std::min(app[0].capacity, app[1].capacity);
    cursor = reinterpret_cast<int64_t*>(S->ctrl + kCurLepton);
  } else {
    a.out_rec[0] = static_cast<Rec<T>*>(app[2].rec);
    a.out_pos[0] = static_cast<T*>(app[2].pos);
    a.out_cap = app[2].capacity;
    cursor = reinterpret_cast<int64_t*>(S->ctrl + kCurPhoton);
  }
  a.counts = S->counts;
  a.offsets = S->offsets;
  a.list = S->list;
  a.list_len = reinterpret_cast<int64_t*>(S->ctrl + kListLen);
  a.queue = reinterpret_cast<unsigned long long*>(S->ctrl + *slot);
  a.stats = reinterpret_cast<unsigned long long*>(S->ctrl + kStats);
  // appended photons with the merge folded in: survivors go to the main photon
  // arrays (the photon count pass uses no work queue, so its first queue word
  // serves as the tile counter)
  const bool fold = merged && photon && !from_main;
  if (fold) {
    a.dst = view_of<T>(ens->s[2]);
    a.dst_cap = ens->s[2].capacity;
    a.dst_cursor = reinterpret_cast<int64_t*>(S->ctrl + kMergedCursor);
    if ((rc = ensure_merged_state(S, (n + kMergedTile - 1) / kMergedTile)) != QED_OK) return rc;
    a.dst_state = S->state_m;
    a.dst_epoch = next_epoch_m(S, st);
    if (!a.dst_epoch) {
      set_error("clearing the look-back words failed");
      return QED_ERR_HIP;
    }
    a.dst_ticket = reinterpret_cast<unsigned long long*>(S->ctrl + *slot);
    a.pair_cursor = reinterpret_cast<int64_t*>(S->ctrl + kCurLepton);
  }
  // leptons: the count pass logs its events and the replay writes from the
  // log (the direct write kernel still runs the launch if the log overflows)
  if (!photon && write_replay_enabled()) {
    if ((rc = ensure_log_heads(S)) != QED_OK) return rc;
    a.log_on = 1;
    a.log_pool = S->log_pool;
    a.log_cap = S->log_pool ? S->log_cap : 0;
    a.log_head = S->log_head;
    a.log_ctl = reinterpret_cast<unsigned long long*>(S->ctrl + *slot + 2 * kQueueWords + 4);
    a.offsets_k = S->offsets_k;
  }
  a.dt = dt;
  a.seed = seed;
  a.step = step;
  a.emission = cfg->emission;
  a.pair = cfg->pair;
  a.push = cfg->push;
  a.positions = positions ? 1 : 0;
  a.write_nev = cfg->nev ? 1 : 0;
  a.gamma_min = cfg->gamma_min;
  a.max_events = cfg->max_events;
  a.tab = tab->view;

  const int p = photon ? 1 : 0;
  size_t lds = sizeof(SrcTable);
  if (sizeof(T) == 4)
    lds += sizeof(float2) * tab->view.rate[p].n +
           sizeof(float) * tab->view.cdf[p].rows32 * tab->view.cdf[p].cols32;
  // leptons: 2 blocks per CU (the emission tables take ~78 KiB of LDS); photons: 4
  const int max_grid = S->num_cu * (photon ? 4 : 2);
  const int grid = (int)std::min<int64_t>((n + kStepThreads - 1) / kStepThreads, max_grid);

  ScanArgs s;
  s.counts = S->counts;
  s.n = n;
  s.offsets = S->offsets;
  s.list = S->list;
  s.cursor = cursor;
  s.list_len = reinterpret_cast<int64_t*>(S->ctrl + kListLen);
  s.state_c = S->state_c;
  s.state_f = S->state_f;
  s.epoch = next_epoch(S, st);
  if (!s.epoch) {
    set_error("clearing the look-back words failed");
    return QED_ERR_HIP;
  }
  s.ticket = reinterpret_cast<unsigned long long*>(S->ctrl + *slot + 2 * kQueueWords);
  s.num_tiles = (n + kScanTile - 1) / kScanTile;
  s.event_particles = reinterpret_cast<unsigned long long*>(S->ctrl + kStats + kStatEventParticles + p);
  s.offsets_k = a.log_on ? S->offsets_k : nullptr;
  *slot += kLaunchWords;

  const int k_count = photon ? 3 : 0, k_write = photon ? 4 : 2;
  hipEvent_t e0 = log.begin();
  hipError_t e = fold     ? launch_count_photon_merged<T>(a, grid, lds, st)
                 : photon ? launch_count<T, true>(a, grid, lds, st)
                          : launch_count<T, false>(a, grid, lds, st);
  if (e != hipSuccess) {
    set_error(std::string("count kernel: ") + hipGetErrorString(e));
    return QED_ERR_HIP;
  }
  log.end(k_count, e0);
  if (!fold) {  // the merged photon pass writes its event list itself
    e0 = log.begin();
    e = launch_scan(s, st);
    if (e != hipSuccess) {
      set_error(std::string("scan kernel: ") + hipGetErrorString(e));
      return QED_ERR_HIP;
    }
    log.end(1, e0);
  }
  e0 = log.begin();
  // The lepton write kernel runs one block per CU.  In FP32 that block has
  // kWriteThreads threads (four waves per SIMD on one copy of the LDS tables)
  // and stages its child records in LDS, written out in half lines, when the
  // slots fit beside the tables.  Otherwise (FP64, or tables too large) it
  // runs kStepThreads threads and stores each record piece by piece.
  const size_t stage_off = line_stage_offset(sizeof(SrcTable), sizeof(T) == 4, tab->view.rate[0].n,
                                             tab->view.cdf[0].rows32 * tab->view.cdf[0].cols32);
  const bool stage = !photon && sizeof(T) == 4 && write_staging_enabled() &&
                     stage_off + kLineStageBytes + kWriteThreads <= kMaxLdsBytes;
  // as many blocks as 512-thread blocks would need, at most one per CU: a
  // small launch still spreads over as many CUs (waves without work leave
  // at once)
  const int wgrid = photon ? grid : (int)std::min<int64_t>((n + kStepThreads - 1) / kStepThreads, S->num_cu);
  // with the event log: the replay (count launch's grid), then the direct
  // write kernel, which returns at once unless the log overflowed
  e = a.log_on ? launch_replay<T>(a, grid, st) : hipSuccess;
  if (e == hipSuccess)
    e = photon ? launch_write<T, true>(a, wgrid, lds, st)
               : launch_write<T, false>(a, wgrid, stage ? stage_off + kLineStageBytes : lds, st, stage);
  if (e != hipSuccess) {
    set_error(std::string("write kernel: ") + hipGetErrorString(e));
    return QED_ERR_HIP;
  }
  log.end(k_write, e0);
  for (int k : {k_count, 1, k_write}) {
    if (k == 1 && fold) continue;
    stats->kernel_launches[k] += 1;
    stats->kernel_particles[k] += device_n ? 0 : n;  // a device-sized range is added after the round
  }
  return QED_OK;
}

// The validation pass: per species, live particles with a non-finite
// momentum, position, weight, optical depth or field component.  Blocking
// (one small device-to-host copy).
template <typename T>
qed_status validate_impl(Scratch* S, const qed_ensemble* ens, int64_t bad[3], hipStream_t st) {
  auto* cnt = reinterpret_cast<unsigned long long*>(S->ctrl + kNonFinite);
  SFQED_HIP(hipMemsetAsync(cnt, 0, 3 * sizeof(uint64_t), st));
  for (int s = 0; s < 3; ++s) {
    const int64_t n = ens->s[s].count;
    SFQED_HIP(launch_count_nonfinite<T>(view_of<T>(ens->s[s]), fields_of<T>(ens->f[s], n), n, cnt + s, st));
  }
  uint64_t h[3];
  const qed_status rb = read_back(S, h, cnt, sizeof(h), st);
  if (rb != QED_OK) return rb;
  for (int s = 0; s < 3; ++s) bad[s] = (int64_t)h[s];
  if (h[0] || h[1] || h[2]) {
    set_error("non-finite values in " + std::to_string(h[0]) + " electrons, " + std::to_string(h[1]) +
              " positrons, " + std::to_string(h[2]) + " photons");
    return QED_ERR_ARG;
  }
  return QED_OK;
}

template <typename T>
qed_status step_impl(const qed_tables* tab, const qed_step_cfg* cfg, qed_ensemble* ens, qed_append* app,
                     double dt, uint64_t seed, uint32_t step, qed_step_stats* stats, hipStream_t st,
                     bool merged = false) {
  Scratch* S = scratch_for_current_device();
  if (!S) {
    set_error("no HIP device");
    return QED_ERR_HIP;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (cfg->validate) {  // before anything is changed
    int64_t bad[3];
    const qed_status v = validate_impl<T>(S, ens, bad, st);
    if (v != QED_OK) return v;
  }
  SFQED_HIP(hipMemsetAsync(S->ctrl, 0, sizeof(uint64_t) * kCtrlWords, st));
  int slot = 0;
  const bool positions = ens->s[0].x != nullptr || ens->s[1].x != nullptr || ens->s[2].x != nullptr;
  qed_step_stats local;
  std::memset(&local, 0, sizeof(local));
  int64_t cur[2] = {0, 0};  // photons, leptons appended so far
  auto read_cursors = [&]() -> qed_status { return read_back(S, cur, S->ctrl + kCurPhoton, sizeof(cur), st); };
  const int64_t capg = app[2].capacity, capl = std::min(app[0].capacity, app[1].capacity);
  EventLog log;
  log.on = cfg->profile != 0;
  log.st = st;
  qed_status rc;
  int64_t launches = 0;
  // one launch per round for the leptons (electrons, then positrons) and per
  // range of photons
  auto launch = [&](int species, bool from_main, int64_t begin0, int64_t n0, int64_t begin1,
                    int64_t n1) -> qed_status {
    if (n0 + n1 <= 0) return QED_OK;
    ++launches;
    return run_launch<T>(S, st, tab, cfg, ens, app, species, from_main, begin0, n0, begin1, n1, dt, seed, step,
                         &slot, positions, log, &local, merged);
  };
  // The photons appended from g_from on, as far as the round's lepton launch
  // got.  qed_step has read the photon cursor back (cur[0]); the merged
  // step's photon pass reads it on the device (one host wait less per round).
  auto launch_appended_photons = [&](int64_t g_from) -> qed_status {
    if (!merged) return launch(2, false, g_from, cur[0] - g_from, 0, 0);
    if (capg - g_from <= 0) return QED_OK;
    ++launches;
    return run_launch<T>(S, st, tab, cfg, ens, app, 2, false, g_from, capg - g_from, 0, 0, dt, seed, step, &slot,
                         positions, log, &local, true, true);
  };
  // after the round's read-back: the appended photons the round processed
  auto photons_done = [&](int64_t g_from) -> int64_t {
    const int64_t g_hi = std::min(cur[0], capg);
    if (merged && g_hi > g_from) {  // a device-sized range: its particles are known only now
      local.kernel_particles[3] += g_hi - g_from;
      local.kernel_particles[4] += g_hi - g_from;
    }
    return g_hi;
  };
  // round 0: the input ensemble, then the photons its leptons emitted
  if ((rc = launch(0, true, 0, ens->s[0].count, 0, ens->s[1].count)) != QED_OK) return rc;
  int64_t g_done = 0;
  bool overflow = false;
  if (!merged) {
    if ((rc = read_cursors()) != QED_OK) return rc;
    overflow = cur[0] > capg;
  }
  if (!overflow) {
    if ((rc = launch(2, true, 0, ens->s[2].count, 0, 0)) != QED_OK) return rc;
    // merged: the input photons are read for the last time in this round, so
    // their survivors are compacted now; appended survivors follow them
    if (merged && ens->s[2].count > 0) {
      const int64_t tiles = (ens->s[2].count + kMergeTile - 1) / kMergeTile;
      if ((rc = ensure_merge_tiles(S, tiles)) != QED_OK) return rc;
      if (slot + kLaunchWords > kSlots) {
        SFQED_HIP(hipMemsetAsync(S->ctrl, 0, sizeof(uint64_t) * kSlots, st));
        slot = 0;
      }
      MergeArgs<T> m;
      m.main = view_of<T>(ens->s[2]);
      m.app = nullptr;
      m.app_pos = nullptr;
      m.n_main = ens->s[2].count;
      m.n_app = 0;
      m.positions = positions ? 1 : 0;
      m.state = S->state_c;
      m.epoch = next_epoch(S, st);
      if (!m.epoch) {
        set_error("clearing the look-back words failed");
        return QED_ERR_HIP;
      }
      m.ticket = reinterpret_cast<unsigned long long*>(S->ctrl + slot);
      m.num_tiles = tiles;
      m.out_count = reinterpret_cast<int64_t*>(S->ctrl + kMergedCursor);
      slot += kLaunchWords;
      SFQED_HIP(launch_merge_photons<T>(m, st));
    }
    if ((rc = launch_appended_photons(0)) != QED_OK) return rc;
    if ((rc = read_cursors()) != QED_OK) return rc;
    g_done = photons_done(0);
    overflow = cur[0] > capg || cur[1] > capl;
  }
  int64_t rounds = 1, l_done = 0;
  while (!overflow && cur[1] > l_done) {
    const int64_t l_hi = cur[1];
    if ((rc = launch(0, false, l_done, l_hi - l_done, l_done, l_hi - l_done)) != QED_OK) return rc;
    l_done = l_hi;
    if (!merged) {
      if ((rc = read_cursors()) != QED_OK) return rc;
      if (cur[0] > capg) {
        overflow = true;
        break;
      }
    }
    if ((rc = launch_appended_photons(g_done)) != QED_OK) return rc;
    if ((rc = read_cursors()) != QED_OK) return rc;
    g_done = photons_done(g_done);
    overflow = cur[0] > capg || cur[1] > capl;
    ++rounds;
  }
  uint64_t dev_stats[8];
  if ((rc = read_back(S, dev_stats, S->ctrl + kStats, sizeof(dev_stats), st)) != QED_OK) return rc;
  grow_log(S, dev_stats[kStatLogNeed]);  // later steps replay launches this one had to re-run
  local.n_emit = cur[0];
  local.n_pair = cur[1];
  local.n_new[0] = cur[1];
  local.n_new[1] = cur[1];
  local.n_new[2] = cur[0];
  local.n_rounds = rounds;
  local.max_events = (int64_t)dev_stats[kStatMaxEvents];
  local.required_capacity[0] = cur[1];
  local.required_capacity[1] = cur[1];
  local.required_capacity[2] = cur[0];
  local.n_launches = launches;
  local.event_particles[0] = (int64_t)dev_stats[kStatEventParticles];
  local.event_particles[1] = (int64_t)dev_stats[kStatEventParticles + 1];
  local.log_replays = (int64_t)dev_stats[kStatReplays];
  local.log_reruns = (int64_t)dev_stats[kStatReruns];
  log.collect(local.kernel_ms);
  app[0].count = std::min(cur[1], app[0].capacity);
  app[1].count = std::min(cur[1], app[1].capacity);
  app[2].count = std::min(cur[0], app[2].capacity);
  if (stats) *stats = local;
  if (overflow) {
    set_error("append capacity exceeded");
    return QED_ERR_CAPACITY;
  }
  if (merged) {
    // the photons are merged; the leptons' records go after the input leptons
    int64_t photons = 0;
    if ((rc = read_back(S, &photons, S->ctrl + kMergedCursor, sizeof(int64_t), st)) != QED_OK) return rc;
    if (ens->s[0].count + app[0].count > ens->s[0].capacity || ens->s[1].count + app[1].count > ens->s[1].capacity ||
        photons > ens->s[2].capacity) {
      ens->s[2].count = std::min(photons, ens->s[2].capacity);
      set_error("merged step: main capacity exceeded (photons " + std::to_string(photons) + ")");
      return QED_ERR_CAPACITY;
    }
    for (int s = 0; s < 2; ++s)
      SFQED_HIP(launch_append_records<T>(view_of<T>(ens->s[s]), ens->s[s].count,
                                         static_cast<const Rec<T>*>(app[s].rec), static_cast<const T*>(app[s].pos),
                                         app[s].count, positions ? 1 : 0, st));
    SFQED_HIP(hipStreamSynchronize(st));
    ens->s[0].count += app[0].count;
    ens->s[1].count += app[1].count;
    ens->s[2].count = photons;
  }
  if (dev_stats[kStatBadRoot]) {
    set_error("an appended record's root names no particle of the ensemble (corrupted append buffer)");
    return QED_ERR_ARG;
  }
  if (dev_stats[kStatCapped]) {
    set_error("a particle reached max_events");
    return QED_ERR_EVENT_CAP;
  }
  return QED_OK;
}

}  // namespace

// The merge on scratch words the caller provides (see MergeScratch in lib.h):
// leptons never die, so their records are appended after the input ensemble;
// photons that died are dropped and the appended survivors follow, one stable
// compaction with a decoupled look-back over tiles of kMergeTile photons.
template <typename T>
qed_status merge_on(qed_ensemble* ens, const qed_append* app, hipStream_t st, const MergeScratch& ms) {
  const bool positions = ens->s[0].x != nullptr || ens->s[1].x != nullptr || ens->s[2].x != nullptr;
  for (int s = 0; s < 2; ++s)
    if (ens->s[s].count + app[s].count > ens->s[s].capacity) {
      set_error("merge: lepton capacity");
      return QED_ERR_CAPACITY;
    }
  const int64_t ntot = ens->s[2].count + app[2].count;
  const int64_t tiles = (ntot + kMergeTile - 1) / kMergeTile;
  if (tiles > ms.tiles) {
    set_error("merge: " + std::to_string(ntot) + " photons exceed the scratch (" + std::to_string(ms.tiles) +
              " tiles of " + std::to_string(kMergeTile) + ")");
    return QED_ERR_CAPACITY;
  }
  // photons: survivors are compacted in place, so they must fit.  When the
  // capacity holds every photon that could survive there is nothing to check;
  // otherwise count the survivors first.
  if (ntot > ens->s[2].capacity) {
    auto* cnt = reinterpret_cast<unsigned long long*>(ms.alive);
    SFQED_HIP(launch_count_alive(ens->s[2].alive, ens->s[2].count, cnt, st));
    SFQED_HIP(launch_count_alive_rec<T>(static_cast<const Rec<T>*>(app[2].rec), app[2].count, cnt, st));
    uint64_t alive_total = 0;
    SFQED_HIP(hipMemcpyAsync(&alive_total, cnt, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    SFQED_HIP(hipStreamSynchronize(st));
    if ((int64_t)alive_total > ens->s[2].capacity) {
      set_error("merge: photon capacity");
      return QED_ERR_CAPACITY;
    }
  }
  for (int s = 0; s < 2; ++s)
    SFQED_HIP(launch_append_records<T>(view_of<T>(ens->s[s]), ens->s[s].count, static_cast<const Rec<T>*>(app[s].rec),
                                       static_cast<const T*>(app[s].pos), app[s].count, positions ? 1 : 0, st));
  int64_t new_photons = 0;
  if (ntot > 0) {
    MergeArgs<T> m;
    m.main = view_of<T>(ens->s[2]);
    m.app = static_cast<const Rec<T>*>(app[2].rec);
    m.app_pos = static_cast<const T*>(app[2].pos);
    m.n_main = ens->s[2].count;
    m.n_app = app[2].count;
    m.positions = positions ? 1 : 0;
    m.state = ms.state;
    m.epoch = ms.epoch;
    m.ticket = reinterpret_cast<unsigned long long*>(ms.ticket);
    m.num_tiles = tiles;
    m.out_count = reinterpret_cast<int64_t*>(ms.count);
    SFQED_HIP(launch_merge_photons<T>(m, st));
    SFQED_HIP(hipMemcpyAsync(&new_photons, ms.count, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  }
  SFQED_HIP(hipStreamSynchronize(st));
  ens->s[0].count += app[0].count;
  ens->s[1].count += app[1].count;
  ens->s[2].count = new_photons;
  return QED_OK;
}
bool merge_args_ok(const qed_ensemble* ens, const qed_append* app) {
  if (!ens || !app || (ens->dtype != QED_F32 && ens->dtype != QED_F64)) {
    set_error("merge: null argument or invalid dtype");
    return false;
  }
  const bool positions = ens->s[0].x != nullptr || ens->s[1].x != nullptr || ens->s[2].x != nullptr;
  for (int s = 0; s < 3; ++s) {
    if (!species_ok(ens->s[s], s == 2, positions) || !append_ok(app[s], positions) || app[s].count < 0 ||
        app[s].count > app[s].capacity) {
      set_error("merge: invalid species " + std::to_string(s));
      return false;
    }
  }
  return true;
}

template qed_status merge_on<float>(qed_ensemble*, const qed_append*, hipStream_t, const MergeScratch&);
template qed_status merge_on<double>(qed_ensemble*, const qed_append*, hipStream_t, const MergeScratch&);

namespace {

template <typename T>
qed_status merge_impl(qed_ensemble* ens, const qed_append* app, hipStream_t st) {
  Scratch* S = scratch_for_current_device();
  if (!S) return QED_ERR_HIP;
  std::lock_guard<std::mutex> lk(S->mu);
  const int64_t tiles = (ens->s[2].count + app[2].count + kMergeTile - 1) / kMergeTile;
  qed_status rc = ensure_merge_tiles(S, tiles);
  if (rc != QED_OK) return rc;
  SFQED_HIP(hipMemsetAsync(S->ctrl, 0, sizeof(uint64_t), st));
  SFQED_HIP(hipMemsetAsync(S->ctrl + kAliveCount, 0, sizeof(uint64_t), st));
  MergeScratch ms;
  ms.state = S->state_c;
  ms.tiles = S->tiles_cap;
  ms.epoch = next_epoch(S, st);
  if (!ms.epoch) {
    set_error("clearing the look-back words failed");
    return QED_ERR_HIP;
  }
  ms.ticket = S->ctrl;
  ms.count = S->ctrl + kMergeCount;
  ms.alive = S->ctrl + kAliveCount;
  return merge_on<T>(ens, app, st, ms);
}

// Resampling after the merge (qed_resample): per species, the leveling
// threshold w_th solves sum_i min(1, w_i / w_th) = target.  F(w) = sum_i
// min(w_i, w) is concave and piecewise linear, so Newton's method on
// F(w) - target w started right of the root (w_0 = sum_i w_i / target) moves
// monotonically left and reaches the root of the piece that holds it: each
// step is w <- S(w) / (target - C(w)), with S the weight below w and C the
// count at or above it; it stops when w no longer decreases.  The passes run
// on the device (k_level_pass keeps the solve's state there): a few are
// queued for every species, the host reads the three states once, and queues
// more only for a solve that has not finished (one pass at a time).  The
// compactions follow, and their counts are read once at the end.
template <typename T>
qed_status resample_impl(qed_ensemble* ens, const qed_resample_cfg* cfg, qed_resample_stats* out, hipStream_t st) {
  Scratch* S = scratch_for_current_device();
  if (!S) return QED_ERR_HIP;
  std::lock_guard<std::mutex> lk(S->mu);
  const size_t part_words = 4 * (size_t)kLevelBlocks;
  if (!S->level) {
    SFQED_HIP(hipMalloc(&S->level, sizeof(double) * 3 * part_words + sizeof(LevelState) * 3));
    SFQED_HIP(hipMemset(S->level, 0, sizeof(double) * 3 * part_words + sizeof(LevelState) * 3));
  }
  LevelState* dstate = reinterpret_cast<LevelState*>(S->level + 3 * part_words);
  const bool positions = ens->s[0].x != nullptr || ens->s[1].x != nullptr || ens->s[2].x != nullptr;
  qed_resample_stats stats;
  std::memset(&stats, 0, sizeof(stats));
  const double e_min2 = cfg->photon_energy_min > 0.0 ? cfg->photon_energy_min * cfg->photon_energy_min : 0.0;
  bool solve[3] = {false, false, false};
  for (int k = 0; k < 3; ++k) {
    const int64_t n = ens->s[k].count;
    stats.count_before[k] = stats.count_after[k] = n;
    const bool filter = k == 2 && e_min2 > 0.0;
    solve[k] = n > 0 && (filter || cfg->target[k] > 0);
    if (!solve[k]) continue;
    const SpeciesView<T> v = view_of<T>(ens->s[k]);
    const int passes = cfg->target[k] > 0 ? 1 + S->level_passes[k] : 1;
    for (int q = 0; q < passes; ++q)
      SFQED_HIP(launch_level_pass<T>(v, n, k == 2 ? 1 : 0, e_min2, cfg->target[k], q == 0 ? 1 : 0,
                                     S->level + k * part_words, dstate + k, st));
  }
  LevelState ls[3];
  qed_status rb = read_back(S, ls, dstate, sizeof(ls), st);
  if (rb != QED_OK) return rb;
  for (int k = 0; k < 3; ++k) {
    if (!solve[k]) continue;
    const SpeciesView<T> v = view_of<T>(ens->s[k]);
    while (!ls[k].done && ls[k].iterations < 100) {
      SFQED_HIP(launch_level_pass<T>(v, ens->s[k].count, k == 2 ? 1 : 0, e_min2, cfg->target[k], 0,
                                     S->level + k * part_words, dstate + k, st));
      if ((rb = read_back(S, &ls[k], dstate + k, sizeof(LevelState), st)) != QED_OK) return rb;
    }
    if (cfg->target[k] > 0) S->level_passes[k] = std::max(2, std::min(kLevelDevicePasses, ls[k].iterations + 1));
  }
  bool compacted[3] = {false, false, false};
  for (int k = 0; k < 3; ++k) {
    if (!solve[k]) continue;
    const int64_t n = ens->s[k].count;
    const bool photon = k == 2, filter = photon && e_min2 > 0.0;
    const int64_t eligible = (int64_t)ls[k].eligible;
    const double wt = ls[k].wt;
    stats.iterations[k] = ls[k].iterations;
    stats.w_threshold[k] = wt;
    if (photon) stats.filtered = n - eligible;
    if (wt <= 0.0 && !(filter && eligible < n)) continue;  // nothing to remove
    const int64_t tiles = (n + kMergeTile - 1) / kMergeTile;
    if (tiles > S->tiles_cap) {
      if (S->state_c) {
        SFQED_HIP(hipDeviceSynchronize());
        (void)hipFree(S->state_c);
        (void)hipFree(S->state_f);
      }
      SFQED_HIP(hipMalloc(&S->state_c, sizeof(uint64_t) * tiles));
      SFQED_HIP(hipMalloc(&S->state_f, sizeof(uint64_t) * tiles));
      SFQED_HIP(hipMemset(S->state_c, 0, sizeof(uint64_t) * tiles));
      SFQED_HIP(hipMemset(S->state_f, 0, sizeof(uint64_t) * tiles));
      S->tiles_cap = tiles;
      S->epoch = 0;
    }
    SFQED_HIP(hipMemsetAsync(S->ctrl, 0, sizeof(uint64_t), st));
    ResampleArgs<T> a;
    a.s = view_of<T>(ens->s[k]);
    a.n = n;
    a.photon = photon ? 1 : 0;
    a.positions = positions ? 1 : 0;
    a.e_min2 = filter ? e_min2 : 0.0;
    a.wt = wt;
    a.seed = cfg->seed;
    a.step = cfg->step;
    a.state = S->state_c;
    a.epoch = next_epoch(S, st);
    if (!a.epoch) {
      set_error("clearing the look-back words failed");
      return QED_ERR_HIP;
    }
    a.ticket = reinterpret_cast<unsigned long long*>(S->ctrl);
    a.num_tiles = tiles;
    a.out_count = reinterpret_cast<int64_t*>(S->ctrl + kResampleCount + k);
    SFQED_HIP(launch_resample<T>(a, st));
    compacted[k] = true;
  }
  if (compacted[0] || compacted[1] || compacted[2]) {
    int64_t kept[3] = {0, 0, 0};
    if ((rb = read_back(S, kept, S->ctrl + kResampleCount, sizeof(kept), st)) != QED_OK) return rb;
    for (int k = 0; k < 3; ++k)
      if (compacted[k]) ens->s[k].count = stats.count_after[k] = kept[k];
  }
  if (out) *out = stats;
  return QED_OK;
}

}  // namespace
}  // namespace sfqed

using namespace sfqed;

extern "C" {

const char* qed_status_str(qed_status s) {
  switch (s) {
    case QED_OK: return "ok";
    case QED_ERR_ARG: return "invalid argument";
    case QED_ERR_CAPACITY: return "capacity exceeded";
    case QED_ERR_HIP: return "HIP runtime error";
    case QED_ERR_STATE: return "invalid state";
    case QED_ERR_EVENT_CAP: return "max_events reached";
  }
  return "unknown status";
}

const char* qed_last_error(void) { return g_error.c_str(); }

int32_t qed_abi_version(void) { return 1; }

void qed_table_cfg_default(qed_table_cfg* c) {
  if (!c) return;
  c->rate_chi_min = 1e-7;
  c->rate_chi_max = 1e5;
  c->rate_nodes = 512;
  c->rad_chi_min = 1e-4;
  c->rad_chi_max = 1e4;
  c->rad_rows = 70;
  c->rad_cols = 265;
  c->rad_x_min = -10.0;
  c->rad_x_max = 23.0;
  c->pair_chi_min = 1e-2;
  c->pair_chi_max = 1e4;
  c->pair_rows = 47;
  c->pair_cols = 185;
  c->pair_x_min = -23.0;
  c->f64_refine = 4;
}

qed_status qed_build_rate_tables(const qed_table_cfg* cfg, void* stream, qed_tables** out) {
  if (!cfg || !out) return QED_ERR_ARG;
  const qed_table_cfg& c = *cfg;
  auto range_ok = [](double lo, double hi) { return finite_pos(lo) && finite_pos(hi) && hi > lo; };
  if (!range_ok(c.rate_chi_min, c.rate_chi_max) || !range_ok(c.rad_chi_min, c.rad_chi_max) ||
      !range_ok(c.pair_chi_min, c.pair_chi_max) || c.rate_chi_max < 1e-3 || c.rate_nodes < 4 ||
      c.rate_nodes > (1 << 16) || c.rad_rows < 4 || c.rad_cols < 4 || c.pair_rows < 4 || c.pair_cols < 4 ||
      !(c.rad_x_max > c.rad_x_min) || !(c.pair_x_min < 0.0) || c.f64_refine < 1 || c.f64_refine > 16) {
    set_error("invalid table configuration");
    return QED_ERR_ARG;
  }
  const size_t lds_rad = sizeof(float2) * c.rate_nodes + sizeof(float) * (size_t)c.rad_rows * c.rad_cols;
  const size_t lds_pair = sizeof(float2) * c.rate_nodes + sizeof(float) * (size_t)c.pair_rows * c.pair_cols;
  if (lds_rad > 96 * 1024 || lds_pair > 96 * 1024) {
    set_error("FP32 tables exceed 96 KiB of LDS");
    return QED_ERR_ARG;
  }
  qed_tables* t = new qed_tables();
  std::memset(t, 0, sizeof(*t));
  (void)hipGetDevice(&t->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  qed_status rc = build_tables(c, st, t);
  if (rc == QED_OK && hipStreamSynchronize(st) != hipSuccess) {
    set_error("table build failed");
    rc = QED_ERR_HIP;
  }
  if (rc != QED_OK) {
    if (t->mem) (void)hipFree(t->mem);
    delete t;
    return rc;
  }
  *out = t;
  return QED_OK;
}

void qed_tables_free(qed_tables* t) {
  if (!t) return;
  if (t->mem) (void)hipFree(t->mem);
  delete t;
}

qed_status qed_tables_export(const qed_tables* t, int which, void* dst, size_t* bytes) {
  if (!t || which < 0 || which > 7 || !bytes) return QED_ERR_ARG;
  const size_t len = t->len[which];
  if (!dst) {
    *bytes = len;
    return QED_OK;
  }
  if (*bytes != len) return QED_ERR_ARG;
  SFQED_HIP(hipMemcpy(dst, static_cast<const char*>(t->mem) + t->off[which], len, hipMemcpyDeviceToHost));
  return QED_OK;
}

qed_status qed_tables_geometry(const qed_tables* t, double* out, int n) {
  // [nseg0, s_lo0, nseg1, s_lo1, herm_n, rows32_0, cols32_0, rows64_0, cols64_0, s0_0, s1_0, x0_0, x1_0,
  //  rows32_1, cols32_1, rows64_1, cols64_1, s0_1, s1_1, x0_1, x1_1]
  if (!t || !out || n < 21) return QED_ERR_ARG;
  const TableGeom& g = t->geom;
  double v[21] = {(double)g.nseg[0], g.cheb_s_lo[0], (double)g.nseg[1], g.cheb_s_lo[1], (double)g.herm_n,
                  (double)g.rows32[0], (double)g.cols32[0], (double)g.rows64[0], (double)g.cols64[0], g.s0[0],
                  g.s1[0], g.x0[0], g.x1[0], (double)g.rows32[1], (double)g.cols32[1], (double)g.rows64[1],
                  (double)g.cols64[1], g.s0[1], g.s1[1], g.x0[1], g.x1[1]};
  std::memcpy(out, v, sizeof(v));
  return QED_OK;
}

void qed_step_cfg_default(qed_step_cfg* c) {
  if (!c) return;
  c->emission = 1;
  c->pair = 1;
  c->push = 1;
  c->gamma_min = 1.0;
  c->max_events = 1 << 20;
  c->profile = 0;
  c->nev = 1;
  c->validate = 0;
}

qed_status qed_init_tau(qed_ensemble* ens, uint64_t seed, uint32_t step, void* stream) {
  if (!ens) return QED_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int s = 0; s < 3; ++s) {
    const qed_species& sp = ens->s[s];
    if (sp.count == 0) continue;
    if (!sp.tau || !sp.id || sp.count < 0) return QED_ERR_ARG;
    SFQED_HIP(launch_init_tau<float>(sp.tau, sp.id, sp.count, seed, step, st));
  }
  return QED_OK;
}

qed_status qed_step(const qed_tables* tab, const qed_step_cfg* cfg, qed_ensemble* ens, qed_append app[3], double dt,
                    uint64_t seed, uint32_t step, qed_step_stats* stats, void* stream) {
  if (!tab || !cfg || !ens || !app) {
    set_error("null argument");
    return QED_ERR_ARG;
  }
  if (!finite_pos(dt) || (ens->dtype != QED_F32 && ens->dtype != QED_F64) || !(cfg->gamma_min >= 1.0) ||
      cfg->max_events < 1) {
    set_error("invalid step configuration");
    return QED_ERR_ARG;
  }
  const bool positions = ens->s[0].x != nullptr || ens->s[1].x != nullptr || ens->s[2].x != nullptr;
  for (int s = 0; s < 3; ++s) {
    if (!species_ok(ens->s[s], s == 2, positions) || !append_ok(app[s], positions)) {
      set_error("invalid species " + std::to_string(s));
      return QED_ERR_ARG;
    }
    if (!fields_ok(ens->f[s], ens->s[s].count)) {
      set_error(fields_error(s));
      return QED_ERR_ARG;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ens->dtype == QED_F32) return step_impl<float>(tab, cfg, ens, app, dt, seed, step, stats, st);
  return step_impl<double>(tab, cfg, ens, app, dt, seed, step, stats, st);
}

qed_status qed_step_merged(const qed_tables* tab, const qed_step_cfg* cfg, qed_ensemble* ens, qed_append app[3],
                           double dt, uint64_t seed, uint32_t step, qed_step_stats* stats, void* stream) {
  if (!tab || !cfg || !ens || !app) {
    set_error("null argument");
    return QED_ERR_ARG;
  }
  if (!finite_pos(dt) || (ens->dtype != QED_F32 && ens->dtype != QED_F64) || !(cfg->gamma_min >= 1.0) ||
      cfg->max_events < 1) {
    set_error("invalid step configuration");
    return QED_ERR_ARG;
  }
  const bool positions = ens->s[0].x != nullptr || ens->s[1].x != nullptr || ens->s[2].x != nullptr;
  for (int s = 0; s < 3; ++s) {
    if (!species_ok(ens->s[s], s == 2, positions) || !append_ok(app[s], positions)) {
      set_error("invalid species " + std::to_string(s));
      return QED_ERR_ARG;
    }
    if (!fields_ok(ens->f[s], ens->s[s].count)) {
      set_error(fields_error(s));
      return QED_ERR_ARG;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ens->dtype == QED_F32) return step_impl<float>(tab, cfg, ens, app, dt, seed, step, stats, st, true);
  return step_impl<double>(tab, cfg, ens, app, dt, seed, step, stats, st, true);
}

qed_status qed_validate(const qed_ensemble* ens, int64_t bad[3], void* stream) {
  if (!ens || (ens->dtype != QED_F32 && ens->dtype != QED_F64)) {
    set_error("null ensemble or bad dtype");
    return QED_ERR_ARG;
  }
  const bool positions = ens->s[0].x != nullptr || ens->s[1].x != nullptr || ens->s[2].x != nullptr;
  for (int s = 0; s < 3; ++s) {
    if (!species_ok(ens->s[s], s == 2, positions)) {
      set_error("invalid species " + std::to_string(s));
      return QED_ERR_ARG;
    }
    if (!fields_ok(ens->f[s], ens->s[s].count)) {
      set_error(fields_error(s));
      return QED_ERR_ARG;
    }
  }
  Scratch* S = scratch_for_current_device();
  if (!S) {
    set_error("no HIP device");
    return QED_ERR_HIP;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  int64_t local[3];
  hipStream_t st = static_cast<hipStream_t>(stream);
  const qed_status rc = ens->dtype == QED_F32 ? validate_impl<float>(S, ens, local, st)
                                              : validate_impl<double>(S, ens, local, st);
  if (bad)
    for (int s = 0; s < 3; ++s) bad[s] = rc == QED_ERR_HIP ? 0 : local[s];
  return rc;
}

qed_status qed_merge(qed_ensemble* ens, const qed_append app[3], void* stream) {
  if (!merge_args_ok(ens, app)) return QED_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ens->dtype == QED_F32) return merge_impl<float>(ens, app, st);
  if (ens->dtype == QED_F64) return merge_impl<double>(ens, app, st);
  return QED_ERR_ARG;
}

void qed_resample_cfg_default(qed_resample_cfg* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
}

qed_status qed_resample(qed_ensemble* ens, const qed_resample_cfg* cfg, qed_resample_stats* stats, void* stream) {
  if (!ens || !cfg) return QED_ERR_ARG;
  if (!(cfg->photon_energy_min >= 0.0) || !std::isfinite(cfg->photon_energy_min)) {
    set_error("resample: photon_energy_min must be finite and >= 0");
    return QED_ERR_ARG;
  }
  const bool positions = ens->s[0].x != nullptr || ens->s[1].x != nullptr || ens->s[2].x != nullptr;
  for (int s = 0; s < 3; ++s) {
    if (cfg->target[s] < 0 || !species_ok(ens->s[s], s == 2, positions)) {
      set_error("resample: invalid species " + std::to_string(s));
      return QED_ERR_ARG;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ens->dtype == QED_F32) return resample_impl<float>(ens, cfg, stats, st);
  if (ens->dtype == QED_F64) return resample_impl<double>(ens, cfg, stats, st);
  return QED_ERR_ARG;
}

qed_status qed_eval_rate(const qed_tables* t, int process, qed_dtype dtype, const void* chi, const void* energy,
                         void* w_out, int64_t n, void* stream) {
  if (!t || (process != 0 && process != 1) || n < 0 || (n > 0 && (!chi || !energy || !w_out))) return QED_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == QED_F32)
    SFQED_HIP(launch_eval_rate<float>(t->view, process, (const float*)chi, (const float*)energy, (float*)w_out, n, st));
  else if (dtype == QED_F64)
    SFQED_HIP(launch_eval_rate<double>(t->view, process, (const double*)chi, (const double*)energy, (double*)w_out, n,
                                       st));
  else
    return QED_ERR_ARG;
  return QED_OK;
}

qed_status qed_eval_particles(const qed_tables* t, int species, qed_dtype dtype, const void* px, const void* py,
                              const void* pz, const qed_fields* f, int64_t n, void* chi_out, void* w_out,
                              void* stream) {
  if (!t || species < 0 || species > 2 || !f || n < 0 || (n > 0 && (!px || !py || !pz || !fields_ok(*f, n))))
    return QED_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == QED_F32)
    SFQED_HIP(launch_eval_particles<float>(t->view, species, (const float*)px, (const float*)py, (const float*)pz,
                                           fields_of<float>(*f, n), n, (float*)chi_out, (float*)w_out, st));
  else if (dtype == QED_F64)
    SFQED_HIP(launch_eval_particles<double>(t->view, species, (const double*)px, (const double*)py,
                                            (const double*)pz, fields_of<double>(*f, n), n, (double*)chi_out,
                                            (double*)w_out, st));
  else
    return QED_ERR_ARG;
  return QED_OK;
}

qed_status qed_sample(const qed_tables* t, int process, qed_dtype dtype, const void* chi, const uint32_t* k,
                      void* out, int64_t n, void* stream) {
  if (!t || (process != 0 && process != 1) || n < 0 || (n > 0 && (!chi || !k || !out))) return QED_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == QED_F32)
    SFQED_HIP(launch_sample<float>(t->view, process, (const float*)chi, k, (float*)out, n, st));
  else if (dtype == QED_F64)
    SFQED_HIP(launch_sample<double>(t->view, process, (const double*)chi, k, (double*)out, n, st));
  else
    return QED_ERR_ARG;
  return QED_OK;
}

}  // extern "C"
