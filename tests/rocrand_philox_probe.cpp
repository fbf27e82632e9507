// Host-only probe: prints rocRAND's Philox4x32-10 block for each
// (seed, subsequence, offset) triple read from stdin.  Used to pin the
// oracle's Philox against an independent implementation.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, sub, off, &st);
    uint4 v = rocrand4(&st);
    std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
