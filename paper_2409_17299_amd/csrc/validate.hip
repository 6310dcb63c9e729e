// validate.hip -- the debug validation pass (qed_validate, and the step's
// `validate` option): per species, the number of live particles whose
// momentum, position, weight or optical depth, or whose field components, are
// not finite.  A NaN or an infinity there would not stop the step: it would
// propagate through chi and the rates into every child of the particle.
#include <hip/hip_runtime.h>

#include "step.h"

namespace sfqed {
namespace {

template <typename T>
__device__ __forceinline__ bool fin3(const T* a, const T* b, const T* c, int64_t i) {
  return __builtin_isfinite(a[i]) && __builtin_isfinite(b[i]) && __builtin_isfinite(c[i]);
}

// One thread per particle (grid-stride); a shared field (stride 0) is read at
// index 0 by every particle, so a bad shared value counts every particle.
template <typename T>
__global__ void k_count_nonfinite(SpeciesView<T> s, FieldView<T> f, int64_t n, unsigned long long* bad) {
  uint32_t c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    bool ok = fin3(s.px, s.py, s.pz, i) && __builtin_isfinite(s.w[i]) && __builtin_isfinite(s.tau[i]);
    if (s.x) ok = ok && fin3(s.x, s.y, s.z, i);
    const int64_t j = i * f.stride;
    ok = ok && fin3(f.ex, f.ey, f.ez, j) && fin3(f.bx, f.by, f.bz, j);
    c += ok ? 0u : 1u;
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(bad, (unsigned long long)c);
}

}  // namespace

template <typename T>
hipError_t launch_count_nonfinite(const SpeciesView<T>& s, const FieldView<T>& f, int64_t n, unsigned long long* bad,
                                  hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t grid = (n + 255) / 256;
  grid = grid > 4096 ? 4096 : grid;
  hipLaunchKernelGGL(k_count_nonfinite<T>, dim3((unsigned)grid), dim3(256), 0, st, s, f, n, bad);
  return hipGetLastError();
}

template hipError_t launch_count_nonfinite<float>(const SpeciesView<float>&, const FieldView<float>&, int64_t,
                                                  unsigned long long*, hipStream_t);
template hipError_t launch_count_nonfinite<double>(const SpeciesView<double>&, const FieldView<double>&, int64_t,
                                                   unsigned long long*, hipStream_t);

}  // namespace sfqed
