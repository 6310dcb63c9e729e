// Prints Philox4x32-10 blocks from rocRAND's host-callable engine for counters
// (id_lo, id_hi, step, j) and key = seed, one line per input line
// "seed id step j" read from stdin.  rocRAND's engine with
// seed(seed, subsequence = step | j << 32, offset = 4 id) starts exactly at that
// counter and key.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
  unsigned long long seed, id, step, j;
  while (std::scanf("%llu %llu %llu %llu", &seed, &id, &step, &j) == 4) {
    rocrand_device::philox4x32_10_engine e(seed, step | (j << 32), 4ull * id);
    uint4 r = e.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
