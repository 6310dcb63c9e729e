// noalloc.hip -- qed_merge_noalloc: the merge (qed_merge) with its scratch in
// a fixed device array, for callers that cannot allocate device memory.
//
// The merge's kernels need look-back words (one per tile of kMergeTile
// photons) and three control words.  qed_merge takes them from the library's
// per-device scratch, which grows with hipMalloc; here they live in
// `scratch`, a file-scope device array of fixed size that every device the
// library runs on holds until the process ends.  The host never passes the
// array's name to a kernel: its device address on each device comes from
// hipGetSymbolAddress, taken once per device with that device current.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "lib.h"
#include "step.h"

namespace sfqed {
namespace {

// Merges of up to kNoAllocTiles tiles of kMergeTile photons (main photons plus
// appended ones before the compaction: 2^17 x 2048 = 268,435,456).
constexpr int64_t kNoAllocTiles = int64_t(1) << 17;
constexpr int64_t kNoAllocCtrl = 32;  // ticket, survivor count, alive count, spare
constexpr int64_t kNoAllocWords = kNoAllocTiles + kNoAllocCtrl;  // 1 MiB + 256 B

static __device__ __align__(256) uint64_t scratch[kNoAllocWords];

__global__ void k_zero_words(uint64_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

hipError_t zero_words(uint64_t* p, int64_t n, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 512);
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

struct DeviceScratch {
  int device = -1;
  uint64_t* ptr = nullptr;  // this device's copy of `scratch`
  uint32_t epoch = 0;       // the last look-back epoch used on it
};
constexpr int kMaxDevices = 64;
std::mutex g_mu;
DeviceScratch g_dev[kMaxDevices];
int g_ndev = 0;

// This device's scratch: the symbol's address is taken the first time the
// device is seen (with it current) and the array is cleared once then.
qed_status device_scratch(hipStream_t st, DeviceScratch** out) {
  int dev = 0;
  SFQED_HIP(hipGetDevice(&dev));
  for (int i = 0; i < g_ndev; ++i)
    if (g_dev[i].device == dev) {
      *out = &g_dev[i];
      return QED_OK;
    }
  if (g_ndev == kMaxDevices) {
    set_error("qed_merge_noalloc: more than 64 devices");
    return QED_ERR_STATE;
  }
  void* p = nullptr;
  SFQED_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  SFQED_HIP(zero_words(static_cast<uint64_t*>(p), kNoAllocWords, st));
  SFQED_HIP(hipStreamSynchronize(st));
  DeviceScratch& d = g_dev[g_ndev++];
  d.device = dev;
  d.ptr = static_cast<uint64_t*>(p);
  d.epoch = 0;
  *out = &d;
  return QED_OK;
}

}  // namespace
}  // namespace sfqed

using namespace sfqed;

extern "C" qed_status qed_merge_noalloc(qed_ensemble* ens, const qed_append app[3], void* stream) {
  if (!merge_args_ok(ens, app)) return QED_ERR_ARG;
  const int64_t ntot = ens->s[2].count + app[2].count;
  if ((ntot + kMergeTile - 1) / kMergeTile > kNoAllocTiles) {
    set_error("qed_merge_noalloc: " + std::to_string(ntot) + " photons before the compaction exceed its limit of " +
              std::to_string(kNoAllocTiles * kMergeTile));
    return QED_ERR_ARG;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceScratch* d = nullptr;
  qed_status rc = device_scratch(st, &d);
  if (rc != QED_OK) return rc;
  // look-back words carry the 24-bit epoch of the merge that wrote them; when
  // the counter wraps they are cleared before epoch 1 is used again
  d->epoch = (d->epoch + 1) & 0xFFFFFFu;
  if (d->epoch == 0) {
    d->epoch = 1;
    SFQED_HIP(zero_words(d->ptr, kNoAllocTiles, st));
  }
  uint64_t* ctrl = d->ptr + kNoAllocTiles;
  SFQED_HIP(zero_words(ctrl, 3, st));  // ticket, survivor count, alive count
  MergeScratch ms;
  ms.state = d->ptr;
  ms.tiles = kNoAllocTiles;
  ms.epoch = d->epoch;
  ms.ticket = ctrl;
  ms.count = ctrl + 1;
  ms.alive = ctrl + 2;
  if (ens->dtype == QED_F32) return merge_on<float>(ens, app, st, ms);
  return merge_on<double>(ens, app, st, ms);
}
