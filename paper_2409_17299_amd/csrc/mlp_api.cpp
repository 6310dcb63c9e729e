// mlp_api.cpp -- C ABI of the inverse-CDF surrogate: parameter upload and
// download, inference, gradients and the Adam training loop.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "lib.h"
#include "mlp.h"

struct qed_mlp {
  int device;
  int num_cu;
  qed_mlp_cfg cfg;
  float* master;   // [kMlpParams]
  float* m;        // Adam first moments
  float* v;        // Adam second moments
  sfqed::MlpPacked* packed;
  float* partial;  // [rows][kGradRow] per-wave partial gradients
  int64_t partial_rows;
  int64_t adam_t;  // Adam steps taken since the last set_params
};

namespace sfqed {
namespace {

bool on_device(const qed_mlp* m) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != m->device) {
    set_error("qed_mlp used with another device current");
    return false;
  }
  return true;
}

MlpGeom geom_of(const qed_mlp_cfg& c) {
  MlpGeom g;
  g.f1_scale = c.f1_scale;
  g.f1_shift = c.f1_shift;
  g.f2_scale = c.f2_scale;
  g.out_scale = c.out_scale;
  g.chi_lo = c.chi_min;
  g.chi_hi = c.chi_max;
  return g;
}

int infer_grid(const qed_mlp* m, int64_t n) {
  const int64_t tiles = (n + 31) / 32;
  const int64_t blocks = (tiles + kMlpThreads / 64 - 1) / (kMlpThreads / 64);
  return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, (int64_t)m->num_cu * 8));
}

// rows of per-wave partial gradients a batch needs (two waves per block)
int64_t grad_rows(int64_t batch) { return ((batch + 63) / 64) * 2; }

qed_status ensure_partial(qed_mlp* m, int64_t batch) {
  const int64_t rows = grad_rows(batch);
  if (rows <= m->partial_rows) return QED_OK;
  if (m->partial) SFQED_HIP(hipFree(m->partial));
  m->partial = nullptr;
  m->partial_rows = 0;
  SFQED_HIP(hipMalloc(&m->partial, sizeof(float) * kGradRow * rows));
  m->partial_rows = rows;
  return QED_OK;
}

bool cfg_ok(const qed_mlp_cfg& c) {
  return std::isfinite(c.chi_min) && std::isfinite(c.chi_max) && c.chi_min > 0.f && c.chi_max >= c.chi_min &&
         std::isfinite(c.f1_scale) && std::isfinite(c.f1_shift) && std::isfinite(c.f2_scale) &&
         std::isfinite(c.out_scale);
}

}  // namespace
}  // namespace sfqed

using namespace sfqed;

extern "C" {

void qed_mlp_cfg_default(qed_mlp_cfg* c) {
  if (!c) return;
  c->chi_min = 1e-2f;
  c->chi_max = 1e2f;
  c->f1_scale = (float)(1.0 / std::log(100.0));
  c->f1_shift = 0.f;
  c->f2_scale = 0.1f;
  c->out_scale = 10.f;
}

void qed_mlp_train_cfg_default(qed_mlp_train_cfg* c) {
  if (!c) return;
  c->steps = 20000;
  c->batch = 16384;
  c->schedule_start = 0;
  c->schedule_len = 0;
  c->lr_max = 3e-3f;
  c->lr_min = 1e-6f;
  c->warmup = 0.05f;
  c->beta1 = 0.9f;
  c->beta2 = 0.999f;
  c->eps = 1e-8f;
  c->seed = 0;
  c->shuffle = 1;
}

qed_status qed_mlp_create(const qed_mlp_cfg* cfg, qed_mlp** out) {
  if (!cfg || !out || !cfg_ok(*cfg)) {
    set_error("invalid surrogate configuration");
    return QED_ERR_ARG;
  }
  qed_mlp* m = new qed_mlp();
  std::memset(m, 0, sizeof(*m));
  m->cfg = *cfg;
  if (hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    set_error("no device");
    return QED_ERR_HIP;
  }
  int v = 0;
  (void)hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, m->device);
  m->num_cu = v > 0 ? v : 1;
  const size_t pb = sizeof(float) * kMlpParams;
  if (hipMalloc(&m->master, pb) != hipSuccess || hipMalloc(&m->m, pb) != hipSuccess ||
      hipMalloc(&m->v, pb) != hipSuccess || hipMalloc(&m->packed, sizeof(MlpPacked)) != hipSuccess ||
      hipMemset(m->master, 0, pb) != hipSuccess || hipMemset(m->m, 0, pb) != hipSuccess ||
      hipMemset(m->v, 0, pb) != hipSuccess || hipMemset(m->packed, 0, sizeof(MlpPacked)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    qed_mlp_free(m);
    set_error("surrogate allocation failed");
    return QED_ERR_HIP;
  }
  *out = m;
  return QED_OK;
}

void qed_mlp_free(qed_mlp* m) {
  if (!m) return;
  (void)hipFree(m->master);
  (void)hipFree(m->m);
  (void)hipFree(m->v);
  (void)hipFree(m->packed);
  (void)hipFree(m->partial);
  delete m;
}

qed_status qed_mlp_get_cfg(const qed_mlp* m, qed_mlp_cfg* cfg) {
  if (!m || !cfg) return QED_ERR_ARG;
  *cfg = m->cfg;
  return QED_OK;
}

qed_status qed_mlp_set_params(qed_mlp* m, const float* params, void* stream) {
  if (!m || !params) return QED_ERR_ARG;
  if (!on_device(m)) return QED_ERR_STATE;
  for (int i = 0; i < kMlpParams; ++i)
    if (!std::isfinite(params[i])) {
      set_error("non-finite parameter");
      return QED_ERR_ARG;
    }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t pb = sizeof(float) * kMlpParams;
  SFQED_HIP(hipMemcpyAsync(m->master, params, pb, hipMemcpyHostToDevice, st));
  SFQED_HIP(hipMemsetAsync(m->m, 0, pb, st));
  SFQED_HIP(hipMemsetAsync(m->v, 0, pb, st));
  SFQED_HIP(launch_mlp_pack(m->master, m->packed, st));
  SFQED_HIP(hipStreamSynchronize(st));
  m->adam_t = 0;
  return QED_OK;
}

qed_status qed_mlp_get_params(const qed_mlp* m, float* params, void* stream) {
  if (!m || !params) return QED_ERR_ARG;
  if (!on_device(m)) return QED_ERR_STATE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  SFQED_HIP(hipMemcpyAsync(params, m->master, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, st));
  SFQED_HIP(hipStreamSynchronize(st));
  return QED_OK;
}

qed_status qed_mlp_forward(const qed_mlp* m, const float* x, float* y, int64_t n, void* stream) {
  if (!m || n < 0 || (n > 0 && (!x || !y))) return QED_ERR_ARG;
  if (!on_device(m)) return QED_ERR_STATE;
  if (n == 0) return QED_OK;
  SFQED_HIP(launch_mlp_forward(m->packed, x, y, n, infer_grid(m, n), static_cast<hipStream_t>(stream)));
  return QED_OK;
}

qed_status qed_mlp_grad(qed_mlp* m, const float* x, const float* t, int64_t n, float* grad, float* loss,
                        void* stream) {
  if (!m || n < 1 || n > (int64_t)1 << 31 || !x || !t || !grad || !loss) return QED_ERR_ARG;
  if (!on_device(m)) return QED_ERR_STATE;
  const qed_status rc = ensure_partial(m, n);
  if (rc != QED_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  SFQED_HIP(launch_mlp_grad(m->packed, x, t, n, n, 0, 0, 0, 0, m->partial, st));
  SFQED_HIP(launch_mlp_reduce(m->partial, (int)grad_rows(n), n, grad, loss, nullptr, nullptr, nullptr, nullptr, 0,
                              AdamArgs{}, st));
  return QED_OK;
}

qed_status qed_mlp_train(qed_mlp* m, const float* x, const float* t, int64_t n, const qed_mlp_train_cfg* cfg,
                         float* loss, void* stream) {
  if (!m || !cfg || !x || !t || n < 1 || n > (int64_t)1 << 32) return QED_ERR_ARG;
  const qed_mlp_train_cfg& c = *cfg;
  const int64_t len = c.schedule_len > 0 ? c.schedule_len : c.steps;
  if (c.steps < 0 || c.batch < 1 || c.batch > n || c.batch > (int64_t)1 << 26 || c.schedule_start < 0 ||
      c.schedule_len < 0 || c.schedule_start + c.steps > std::max<int64_t>(len, c.steps) || !(c.lr_max >= 0.f) ||
      !(c.lr_min >= 0.f) || !(c.warmup >= 0.f && c.warmup <= 1.f) || !(c.beta1 >= 0.f && c.beta1 < 1.f) ||
      !(c.beta2 >= 0.f && c.beta2 < 1.f) || !(c.eps > 0.f)) {
    set_error("invalid training configuration");
    return QED_ERR_ARG;
  }
  if (!on_device(m)) return QED_ERR_STATE;
  const qed_status rc = ensure_partial(m, c.batch);
  if (rc != QED_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int rows = (int)grad_rows(c.batch);
  const int64_t warm = std::max<int64_t>(1, (int64_t)std::llround((double)c.warmup * (double)len));
  for (int64_t i = 0; i < c.steps; ++i) {
    const int64_t s = c.schedule_start + i;  // position in the schedule
    double lr;
    if (s < warm) {
      lr = c.lr_max * (double)(s + 1) / (double)warm;
    } else {
      const double span = (double)std::max<int64_t>(1, len - warm);
      lr = c.lr_min + 0.5 * (c.lr_max - c.lr_min) * (1.0 + std::cos(M_PI * (double)(s - warm) / span));
    }
    ++m->adam_t;
    AdamArgs a;
    a.lr = (float)lr;
    a.beta1 = c.beta1;
    a.beta2 = c.beta2;
    a.eps = c.eps;
    a.bc1 = (float)(1.0 - std::pow((double)c.beta1, (double)m->adam_t));
    a.bc2 = (float)(1.0 - std::pow((double)c.beta2, (double)m->adam_t));
    // consecutive batches: the schedule step's window, wrapping around the data
    const int64_t base = (int64_t)(((unsigned __int128)s * (unsigned __int128)c.batch) % (unsigned __int128)n);
    SFQED_HIP(launch_mlp_grad(m->packed, x, t, n, c.batch, base, c.shuffle ? 1 : 0, c.seed, (uint32_t)s,
                              m->partial, st));
    SFQED_HIP(launch_mlp_reduce(m->partial, rows, c.batch, nullptr, loss ? loss + i : nullptr, m->master, m->m,
                                m->v, m->packed, 1, a, st));
  }
  return QED_OK;
}

qed_status qed_sample_mlp(const qed_tables* t, const qed_mlp* m, const float* chi, const uint32_t* k, float* delta,
                          int64_t n, void* stream) {
  if (!t || !m || n < 0 || (n > 0 && (!chi || !k || !delta))) return QED_ERR_ARG;
  if (!on_device(m)) return QED_ERR_STATE;
  if (n == 0) return QED_OK;
  SFQED_HIP(launch_mlp_sample(m->packed, geom_of(m->cfg), t->view, chi, k, delta, n, infer_grid(m, n),
                              static_cast<hipStream_t>(stream)));
  return QED_OK;
}

}  // extern "C"
