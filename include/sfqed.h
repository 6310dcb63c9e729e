/* sfqed.h -- C ABI of libsfqed, the MI355X (gfx950) per-macroparticle
 * strong-field QED event generator.
 *
 * The library implements the inverse-sampling generator with sub-cycling of
 * arXiv:2409.17299 (Sec. 3, Algorithms 1 and 2): for every electron, positron
 * and photon it evaluates the quantum parameter chi, the locally-constant-field
 * emission or pair rate from precomputed tables, carries an FP64 optical depth
 * across sub-cycles, samples the energy fraction of each new particle by
 * inverse CDF, applies collinear recoil and appends the new photons and pairs
 * in a deterministic order.  New particles are advanced to the end of the same
 * global step (Algorithm 2).
 *
 * Units throughout: momenta in m_e c; E in E_S = m_e^2 c^3/(e hbar); B in
 * E_S / c; times in hbar/(m_e c^2); lengths in hbar/(m_e c).
 *
 * Memory: every particle and field array is a device pointer owned by the
 * caller (for example torch tensors); tables and surrogate networks are owned
 * by the library.  All calls are ordered on the HIP stream passed as
 * `stream` (NULL = the null stream).  Calls that read counts back wait for
 * that stream: qed_step and qed_step_merged once per generation round (the
 * append counters), qed_merge and qed_resample at their end (the new counts),
 * qed_build_rate_tables and qed_mlp_set_params / qed_mlp_get_params once.
 * The others only queue work.
 *
 * Concurrency: the library keeps one set of counters and look-back words per
 * device and reuses it in every call on that device.  Calls on one device must
 * therefore not overlap on the GPU: issue them on one stream, or synchronise
 * before switching streams.
 *
 * Library scratch: qed_step and qed_step_merged keep per-device scratch in
 * library-owned device memory that grows (hipMalloc) to the largest launch
 * so far: per-particle counts and offsets, and the event log of the lepton
 * count pass, which the write pass replays.  After a step the log grows to
 * 5/4 of what the step needed, as long as that is at most half of the free
 * device memory; launches whose log does not fit are written by re-running
 * their event loop instead (the same results).  The scratch lives until the
 * process ends.
 *
 * Environment: SFQED_WRITE_STAGING=0 makes the FP32 step store each child
 * record directly instead of staging it in LDS; SFQED_WRITE_REPLAY=0 turns
 * the event log off (the write pass re-runs every event loop).  Both give the
 * same results, slower; they exist so that the paths can be compared.
 *
 * Errors: every function returns a qed_status and never aborts.  Invalid
 * arguments are rejected before any work is queued.
 */
#ifndef SFQED_H
#define SFQED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QED_OK = 0,
  QED_ERR_ARG = 1,       /* bad pointer, size, dtype or configuration */
  QED_ERR_CAPACITY = 2,  /* an append or merge target is too small; see qed_step_stats */
  QED_ERR_HIP = 3,       /* a HIP runtime call failed */
  QED_ERR_STATE = 4,     /* object not built / wrong object kind */
  QED_ERR_EVENT_CAP = 5  /* a particle reached max_events in one step */
} qed_status;

typedef enum { QED_F32 = 0, QED_F64 = 1 } qed_dtype;
enum { QED_ELECTRON = 0, QED_POSITRON = 1, QED_PHOTON = 2 };
enum { QED_EMISSION = 0, QED_PAIR = 1 };

/* ------------------------------------------------------------------ tables
 * Rates (Sec. 3: one rate evaluation per event or per global step) and
 * inverse CDFs (Sec. 3: two-dimensional look-up tables in energy fraction and
 * chi) of nonlinear Compton emission and Breit-Wheeler pair production in the
 * locally-constant-field approximation, built on the GPU in FP64 by quadrature
 * of the modified-Bessel spectra.
 *  - FP64 rates: piecewise Chebyshev (degree 16, segments of 0.5 in ln chi)
 *    of g(s) = ln(W gamma / (alpha chi)) (emission) and
 *    ln(W eps/(alpha chi)) + 8/(3 chi) (pairs) over [rate_chi_min, rate_chi_max].
 *  - FP32 rates: cubic Hermite of the same g on rate_nodes uniform nodes.
 *  - Above the tables (chi beyond the last Chebyshev segment, at least
 *    rate_chi_max) both rates follow their chi^(2/3) limits as
 *    exp(a chi^(-2/3)), a matched at the last node: within 2e-7 of the
 *    quadrature up to chi = 1e10.  Below rate_chi_min emission uses the
 *    classical series and pairs are zero.
 *  - Inverse CDFs: q = logit(delta) - ln chi (emission) and q = logit(xi)
 *    (pairs, xi <= 1/2 tabulated, the rest by symmetry) on a uniform grid in
 *    (ln chi, logit r); FP32 grids are staged in LDS by the step kernels, FP64
 *    grids are f64_refine times finer in both directions and stay in HBM.
 */
typedef struct {
  double rate_chi_min, rate_chi_max; /* FP64 Chebyshev and FP32 Hermite range */
  int32_t rate_nodes;                /* FP32 Hermite nodes */
  double rad_chi_min, rad_chi_max;   /* emission inverse-CDF chi range */
  int32_t rad_rows, rad_cols;        /* FP32 emission grid (ln chi x logit r) */
  double rad_x_min, rad_x_max;       /* logit r range of the emission grid */
  double pair_chi_min, pair_chi_max; /* pair inverse-CDF chi range */
  int32_t pair_rows, pair_cols;      /* FP32 pair grid; logit r in [pair_x_min, 0] */
  double pair_x_min;
  int32_t f64_refine;                /* FP64 grids: (rows-1)*k+1 x (cols-1)*k+1 */
} qed_table_cfg;

typedef struct qed_tables qed_tables; /* opaque, library-owned device memory */

/* Fills cfg with the defaults (rates on [1e-7, 1e5], emission CDF on
 * [1e-4, 1e4] x [-10, 23] with 72 x 265 nodes, pair CDF on [1e-2, 1e4] x
 * [-23, 0] with 47 x 185 nodes, FP64 refinement 4). */
void qed_table_cfg_default(qed_table_cfg *cfg);

/* Builds all tables on the device of the current HIP context, ordered on
 * `stream`; *out receives the handle.  Returns QED_ERR_ARG for an invalid
 * cfg (ranges must be positive and increasing, grids >= 4 nodes, the FP32
 * emission grid must fit in 96 KiB of LDS). */
qed_status qed_build_rate_tables(const qed_table_cfg *cfg, void *stream, qed_tables **out);
void qed_tables_free(qed_tables *t);

/* Table export for validation.  which: 0 emission Chebyshev coefficients,
 * 1 pair Chebyshev coefficients (double [segments][17]), 2 emission FP32
 * Hermite (float [nodes][2]: g, h g'), 3 pair FP32 Hermite, 4 emission FP32
 * inverse CDF (float [rows][cols]), 5 pair FP32 inverse CDF, 6 emission FP64
 * inverse CDF (double), 7 pair FP64 inverse CDF.  *bytes receives the size
 * when dst is NULL; otherwise exactly that many bytes are copied (blocking). */
qed_status qed_tables_export(const qed_tables *t, int which, void *dst, size_t *bytes);

/* ------------------------------------------------------------------ particles
 * The input ensemble: one species as a structure of arrays, caller-owned
 * device pointers.  Momenta and positions have the step's dtype.  x, y, z may
 * all be NULL (positions not advanced).  alive is required for photons (a
 * photon that produced a pair is marked 0) and ignored for leptons.  nev
 * (optional) receives each particle's number of events in the last step. */
typedef struct {
  void *px, *py, *pz;
  void *x, *y, *z;
  float *w;
  double *tau;
  uint64_t *id;
  uint8_t *alive;
  int32_t *nev;
  int64_t count, capacity;
} qed_species;

/* Appended particles: one 16-byte-aligned record per particle, written with
 * full 16-byte stores (the children of one parent are contiguous records).
 * root = species << 30 | index of the input particle whose fields the record
 * sees; t_birth is the time within the step at which it was created; nev is
 * its number of events (written when qed_step_cfg.nev is set); alive is 0 for
 * a photon that produced a pair.  FP32 steps use qed_rec32 (48 bytes), FP64
 * steps qed_rec64 (64 bytes). */
typedef struct {
  float px, py, pz, t_birth;
  double tau;
  uint64_t id;
  float w;
  uint32_t root;
  int32_t nev;
  uint32_t alive;
} qed_rec32;

typedef struct {
  double px, py, pz, t_birth;
  double tau;
  uint64_t id;
  float w;
  uint32_t root;
  int32_t nev;
  uint32_t alive;
} qed_rec64;

/* One species of appended particles: `rec` holds capacity records; `pos`
 * (NULL unless positions are advanced) holds x, y, z, unused per record in the
 * step's dtype.  count is set by qed_step. */
typedef struct {
  void *rec;
  void *pos;
  int64_t count, capacity;
} qed_append;

/* Per-particle fields of one species (dtype of the step), indexed like the
 * particles when stride = 1, or one shared value when stride = 0.  n: entries
 * per array; with stride = 1 it must be at least the species' count (the
 * entry points that take fields return QED_ERR_ARG otherwise, before any
 * device work); ignored with stride = 0. */
typedef struct {
  const void *ex, *ey, *ez, *bx, *by, *bz;
  int64_t stride;
  int64_t n;
} qed_fields;

typedef struct {
  qed_dtype dtype;
  qed_species s[3]; /* QED_ELECTRON, QED_POSITRON, QED_PHOTON */
  qed_fields f[3];
} qed_ensemble;

/* The step samples energy fractions from the inverse-CDF tables.  The
 * learned surrogate (qed_sample_mlp below) is a standalone sampler: on this
 * chip it is several times slower than the FP32 table, and inside the step
 * each loop trip would have to evaluate the network for the whole wave. */
typedef struct {
  int32_t emission, pair, push; /* processes on/off; push: Boris between events */
  double gamma_min;             /* leptons with gamma < gamma_min do not emit (>= 1) */
  int64_t max_events;           /* per particle and step; reaching it is an error */
  int32_t profile;              /* 1: time every launch with HIP events into stats */
  int32_t nev;                  /* 1: write event counts (nev) of appended particles */
  int32_t validate;             /* 1: run qed_validate first; on QED_ERR_ARG nothing is changed */
} qed_step_cfg;

void qed_step_cfg_default(qed_step_cfg *cfg);

typedef struct {
  int64_t n_emit, n_pair;           /* events of the step */
  int64_t n_new[3];                 /* particles appended per species */
  int64_t n_rounds;                 /* generation rounds (Algorithm 2 loop trips) */
  int64_t max_events;               /* largest number of events of one particle */
  int64_t required_capacity[3];     /* append sizes needed (lower bound on overflow) */
  int64_t n_launches;               /* particle-range launches (count, scan, write each) */
  /* Per kernel, indexed 0 count (leptons), 1 scan, 2 write (leptons),
   * 3 count (photons), 4 write (photons).  kernel_ms needs profile = 1 (HIP
   * events on the step's stream, read after the step; no extra waits). */
  double kernel_ms[5];
  int64_t kernel_launches[5];
  int64_t kernel_particles[5];      /* particles in the launches' ranges */
  int64_t event_particles[2];       /* particles with events: leptons, photons */
  int64_t log_replays;              /* lepton launches written from the count pass's event log */
  int64_t log_reruns;               /* lepton launches whose log did not fit (tables re-run) */
} qed_step_stats;

/* Draws tau = -ln(u) for every particle with tau < 0 (u from Philox4x32-10,
 * key = seed, counter = (id_lo, id_hi, step, 0xFFFFFFFF)). */
qed_status qed_init_tau(qed_ensemble *ens, uint64_t seed, uint32_t step, void *stream);

/* One global step of length dt (Algorithms 1 and 2).  Every particle of `ens`
 * is advanced from t = 0 to dt; new particles are appended to `app` (counts
 * start from zero) and advanced from their birth time to dt in later rounds.
 * Momenta, positions, tau and nev of `ens` and `app` are updated in place;
 * photons that produced a pair get alive = 0.  Random draws: Philox4x32-10,
 * key = seed, counter = (id_lo, id_hi, step, j) for the j-th event of a
 * particle in the step; the ids of new particles come from counter word
 * j | 0x80000000.  Order of `app`: creation rounds in order; within a round
 * electrons, then positrons, then photons are processed in index order and
 * each one's children are appended in event order.
 * On QED_ERR_CAPACITY nothing is written past any capacity and
 * stats->required_capacity tells how much would have been needed; the
 * ensemble is then partly advanced and the caller restores it. */
qed_status qed_step(const qed_tables *tab, const qed_step_cfg *cfg, qed_ensemble *ens, qed_append app[3],
                    double dt, uint64_t seed, uint32_t step, qed_step_stats *stats, void *stream);

/* Debug validation pass.  Counts, per species, the live particles (index <
 * count) whose momentum, position (when present), weight or optical depth, or
 * whose six field components (the particle's own, or the shared value when
 * stride = 0), are not finite: a NaN or an infinity there does not stop the
 * step but spreads through chi and the rates into every child of the
 * particle.  bad (may be NULL) receives the three counts.  Returns QED_ERR_ARG
 * when any count is non-zero (qed_last_error names them), QED_OK otherwise.
 * It reads each live particle once and waits for `stream` (one small
 * device-to-host copy); qed_step_cfg.validate = 1 runs it at the start of
 * qed_step and qed_step_merged, before anything is changed. */
qed_status qed_validate(const qed_ensemble *ens, int64_t bad[3], void *stream);

/* Merge (the merge of per-thread arrays of Sec. 4.2): drops photons with
 * alive = 0 from `ens` (stable), then appends the surviving particles of
 * `app` after each species, converting records to the ensemble's arrays.
 * Capacity of ens->s[k] must hold the result, otherwise QED_ERR_CAPACITY and
 * nothing is changed.  ens->s[k].count is updated (blocking: one small
 * device-to-host copy). */
qed_status qed_merge(qed_ensemble *ens, const qed_append app[3], void *stream);

/* qed_merge for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same merge, with the same results and errors, whose look-back words and
 * counters live in a fixed array of 1 MiB + 256 B in the library's device
 * memory instead of its growing scratch.  The array is set up (its address
 * taken and cleared) on the first call on each device and every device the
 * library runs on keeps it until the process ends.  It calls no hipMalloc or
 * hipFree.  Limit: ens->s[2].count + app[2].count <= 268,435,456 photons
 * (2^17 tiles of 2048), else QED_ERR_ARG before any work.  All calls on one
 * device share its array: calls that overlap on one GPU race (issue them on
 * one stream, or synchronise between them).  Blocking like qed_merge. */
qed_status qed_merge_noalloc(qed_ensemble *ens, const qed_append app[3], void *stream);

/* qed_step followed by qed_merge, with the photons merged inside the step
 * (Algorithm 2, then the merge of Sec. 4.2): the input photons are compacted
 * once their round is done, and every appended photon that survives the step
 * is written straight into ens->s[2] by the pass that decides it has no pair
 * event, instead of being read back from its record by the merge.  The
 * resulting ensemble (arrays, order, counts) is identical to qed_step then
 * qed_merge; app[0..1] and app[2] hold the appended records as qed_step
 * leaves them, except that app[2]'s records keep the state the photons were
 * emitted with (their final states are in ens->s[2]).  Capacity of ens->s[k]
 * must hold the merged result: on QED_ERR_CAPACITY nothing is written past
 * it and the ensemble is partly advanced (the caller restores it). */
qed_status qed_step_merged(const qed_tables *tab, const qed_step_cfg *cfg, qed_ensemble *ens, qed_append app[3],
                           double dt, uint64_t seed, uint32_t step, qed_step_stats *stats, void *stream);

/* Resampling after the merge.  Sec. 4.2 notes that photons too soft ever to
 * produce a pair need not join the ensemble, and Sec. 5.1 keeps the cascade's
 * number of macroparticles in check with "global leveling" resampling.
 *   photon_energy_min: photons with |k|^2 < photon_energy_min^2 (FP64) are
 *     removed; 0 removes none (2 removes those below the pair threshold);
 *   target[k]: when species k, after the filter, holds more than target[k]
 *     particles, it is thinned with one threshold weight w_th solving
 *     sum_i min(1, w_i / w_th) = target[k]: a particle with w >= w_th stays
 *     as it is, a lighter one stays when its draw u < w / w_th and then
 *     weighs w_th (every particle keeps its expected weight).  0: no thinning;
 *   draws: u = (x + 1/2) 2^-32, x the first word of Philox4x32-10 with
 *     key = seed and counter (id_lo, id_hi, step, 0xFFFFFFFD).
 * Survivors keep their order, in place; ens->s[k].count is updated; nev is
 * not carried.  Blocking (small device-to-host copies for the threshold). */
typedef struct {
  double photon_energy_min;
  int64_t target[3];
  uint64_t seed;
  uint32_t step;
} qed_resample_cfg;

typedef struct {
  int64_t count_before[3], count_after[3];
  int64_t filtered;        /* photons removed by the energy filter */
  double w_threshold[3];   /* leveling threshold weight; 0 where the species was not thinned */
  int32_t iterations[3];   /* passes of the threshold solve */
} qed_resample_stats;

void qed_resample_cfg_default(qed_resample_cfg *cfg);  /* no filter, no thinning, seed 0, step 0 */
qed_status qed_resample(qed_ensemble *ens, const qed_resample_cfg *cfg, qed_resample_stats *stats, void *stream);

/* ------------------------------------------------------------------ grid fields
 * Given fields on a grid, the field stage in front of the QED step of a PIC
 * code (Sec. 5.1: the test problem is a plane wave in a periodic box, with
 * fields homogeneous across the x axis, so one line of nodes along x holds
 * them).  Units as everywhere: x in hbar / (m_e c), fields in units of the
 * Schwinger field.
 *
 * qed_grid1d: nx nodes at x_i = x0 + i dx, dx = length / nx, periodic with
 * period `length`; each node holds all six components (collocated), nx values
 * per device array, in `dtype`. */
typedef struct {
  qed_dtype dtype;
  int64_t nx;
  double x0, length;
  void *ex, *ey, *ez, *bx, *by, *bz;
} qed_grid1d;

/* Fills the nodes with the standing circularly polarised wave of Sec. 5.1:
 * with phi = k (x_i - xc),
 *   E = e0 cos(phi) (0, cos(omega t), sin(omega t)),
 *   B = e0 sin(phi) (0, cos(omega t), sin(omega t)),
 * two counter-propagating circularly polarised waves of amplitude e0 / 2 whose
 * electric field rotates in the y-z plane, with its antinode at xc (a solution
 * of Maxwell's equations for omega = k).  Evaluated in FP64 (device sin and
 * cos), rounded once to dtype.  Asynchronous on `stream`. */
qed_status qed_grid_standing_wave(const qed_grid1d *g, double e0, double k, double omega, double xc, double t,
                                  void *stream);

/* Periodic box: axis a wraps into [lo[a], lo[a] + len[a]); len[a] = 0 leaves
 * the axis unwrapped. */
typedef struct {
  double lo[3], len[3];
} qed_box;

/* Per-particle field arrays written by qed_gather_fields (dtype of the
 * ensemble); n: entries per array, at least the species' count (else
 * QED_ERR_ARG before any device work).  Pass them to qed_step as a
 * qed_fields with stride 1 and the same n. */
typedef struct {
  void *ex, *ey, *ez, *bx, *by, *bz;
  int64_t n;
} qed_field_arrays;

/* For every particle of the three species of `ens` (positions required):
 * 1. wraps each coordinate into the box (FP64, no fused operations):
 *      s = floor((x - lo) * (1 / len)),  x' = x - s * len,
 *      x' < lo: x' += len;  x' >= lo + len: x' -= len,
 *    and stores x' rounded to dtype (a coordinate is written only when that
 *    changes it);
 * 2. interpolates the grid linearly at the stored x (FP64, no fused operations):
 *      u = (x - x0) * (nx / length),  q = floor(u),  f = u - q,
 *      i = q - nx floor(q / nx) (clamped to [0, nx - 1]),  j = (i + 1) mod nx,
 *      field = (1 - f) g[i] + f g[j],
 *    rounded to dtype, into out[s].
 * The reciprocals 1 / len and nx / length are rounded once.  The grid's dtype
 * must be the ensemble's.  Returns QED_ERR_ARG for a missing array, a
 * non-finite or negative box length, or nx < 1.  Asynchronous on `stream`. */
qed_status qed_gather_fields(qed_ensemble *ens, const qed_grid1d *g, const qed_box *box,
                             const qed_field_arrays out[3], void *stream);

/* ------------------------------------------------------------------ kernels of the step, exposed for validation
 * Rates W (per unit time) of one process for given chi and energy (gamma for
 * emission, eps for pairs), evaluated exactly as inside qed_step (FP64:
 * Chebyshev; FP32: Hermite), in dtype.  Pairs below eps = 2 are not masked
 * here (qed_eval_particles does). */
qed_status qed_eval_rate(const qed_tables *t, int process, qed_dtype dtype, const void *chi, const void *energy,
                         void *w_out, int64_t n, void *stream);

/* chi and rate of each particle of one species (dtype arrays, fields with stride). */
qed_status qed_eval_particles(const qed_tables *t, int species, qed_dtype dtype, const void *px, const void *py,
                              const void *pz, const qed_fields *f, int64_t n, void *chi_out, void *w_out,
                              void *stream);

/* Inverse-CDF samples: out = delta (emission) or xi (pairs) for chi and raw
 * 32-bit uniforms k (r = (k + 1/2) / 2^32). */
qed_status qed_sample(const qed_tables *t, int process, qed_dtype dtype, const void *chi, const uint32_t *k,
                      void *out, int64_t n, void *stream);

/* ------------------------------------------------------------------ surrogate
 * A learned replacement of the emission inverse CDF (the two-dimensional table
 * in chi and energy fraction of Sec. 3): a 2 -> 64 -> 64 -> 1 perceptron with
 * SiLU activations maps x1 = ln(chi) f1_scale + f1_shift and x2 = logit(r)
 * f2_scale to y, and delta = sigmoid(out_scale y + ln chi).  Layer 2 (and its
 * backward) multiplies BF16 weights by BF16 activations with FP32
 * accumulation (MFMA); layers 1 and 3 are FP32.  Inside [chi_min, chi_max] the
 * network samples; outside it the FP32 table does (the fallback).
 *
 * Parameters are 4417 FP32 numbers in the order W1[64][2], b1[64],
 * W2[64][64] (row = output), b2[64], w3[64], b3.  Training minimises the mean
 * squared error of y against targets with Adam (FP32 master weights, FP32
 * moments), entirely on the device; per-wave partial gradients are summed in a
 * fixed order, so results do not depend on scheduling.
 * A qed_mlp belongs to the device current at qed_mlp_create; its calls must
 * run with that device current.  Calls that overlap on one qed_mlp race. */
#define QED_MLP_PARAMS 4417
typedef struct qed_mlp qed_mlp;

typedef struct {
  float chi_min, chi_max;     /* trained range (the table samples outside) */
  float f1_scale, f1_shift;   /* x1 = ln(chi) f1_scale + f1_shift */
  float f2_scale;             /* x2 = logit(r) f2_scale */
  float out_scale;            /* q = out_scale y = logit(delta) - ln chi */
} qed_mlp_cfg;

/* chi in [1e-2, 1e2], x1 = ln chi / ln 100, x2 = logit(r) / 10, q = 10 y. */
void qed_mlp_cfg_default(qed_mlp_cfg *cfg);

/* Allocates the network (all parameters zero) on the current device. */
qed_status qed_mlp_create(const qed_mlp_cfg *cfg, qed_mlp **out);
void qed_mlp_free(qed_mlp *m);
qed_status qed_mlp_get_cfg(const qed_mlp *m, qed_mlp_cfg *cfg);

/* Host copies of the FP32 parameters (QED_MLP_PARAMS floats).  set also
 * resets the Adam moments and step count.  Both wait for the stream. */
qed_status qed_mlp_set_params(qed_mlp *m, const float *params, void *stream);
qed_status qed_mlp_get_params(const qed_mlp *m, float *params, void *stream);

/* y[i] = network output for inputs x[i] = (x1, x2); device arrays x [n][2]
 * and y [n]. */
qed_status qed_mlp_forward(const qed_mlp *m, const float *x, float *y, int64_t n, void *stream);

/* Gradient (device, QED_MLP_PARAMS floats, parameter order) and value (device,
 * one float) of L = mean over i of (y(x_i) - t_i)^2, for device arrays
 * x [n][2] and t [n]; n >= 1. */
qed_status qed_mlp_grad(qed_mlp *m, const float *x, const float *t, int64_t n, float *grad, float *loss,
                        void *stream);

typedef struct {
  int64_t steps, batch;       /* Adam steps of this call and samples per step (batch <= n) */
  int64_t schedule_start;     /* index of this call's first step in the schedule (for chunked runs) */
  int64_t schedule_len;       /* length of the schedule; 0: steps */
  float lr_max, lr_min;       /* linear warm-up to lr_max over warmup * schedule_len, then cosine to lr_min */
  float warmup;
  float beta1, beta2, eps;
  uint64_t seed;              /* batch sampling (Philox, counter = schedule step) */
  int32_t shuffle;            /* 1: batches of independent uniform draws of the data index;
                                 0: consecutive batches cycling through the data in order */
} qed_mlp_train_cfg;

void qed_mlp_train_cfg_default(qed_mlp_train_cfg *cfg);

/* Trains on device data x [n][2], t [n]: `steps` Adam steps continuing from
 * the current parameters and moments.  loss (device, steps floats, or NULL)
 * receives each step's batch loss before its update.  Asynchronous on the
 * stream; the network's scratch grows with the batch (hipMalloc). */
qed_status qed_mlp_train(qed_mlp *m, const float *x, const float *t, int64_t n, const qed_mlp_train_cfg *cfg,
                         float *loss, void *stream);

/* Emission energy fractions delta (FP32, device) for chi and raw uniforms k
 * (r = (k + 1/2) / 2^32): the network inside its chi range, the FP32 table of
 * `t` outside it. */
qed_status qed_sample_mlp(const qed_tables *t, const qed_mlp *m, const float *chi, const uint32_t *k, float *delta,
                          int64_t n, void *stream);

/* Grid geometry of built tables (21 doubles): nseg_rad, s_lo_rad, nseg_pair,
 * s_lo_pair, hermite_nodes, then per process (emission, pairs): rows32,
 * cols32, rows64, cols64, s_first, s_last, x_first, x_last. */
qed_status qed_tables_geometry(const qed_tables *t, double *out, int n);

const char *qed_status_str(qed_status s);
/* Message of the last failure on the calling thread (empty if none). */
const char *qed_last_error(void);
int32_t qed_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SFQED_H */
