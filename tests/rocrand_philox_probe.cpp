// Independent Philox4x32-10 reference for the oracle's tests: runs rocRAND's
// host-side Philox engine (header-only; no GPU needed) and prints the 32-bit
// words of `count` consecutive counters starting at subsequence `subseq`.
// Usage: probe <seed (decimal)> <subsequence> <count>
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  if (argc != 4) return 2;
  unsigned long long seed = std::strtoull(argv[1], nullptr, 10);
  unsigned long long subseq = std::strtoull(argv[2], nullptr, 10);
  long count = std::strtol(argv[3], nullptr, 10);
  rocrand_state_philox4x32_10 st;
  rocrand_init(seed, subseq, 0, &st);
  for (long i = 0; i < count; ++i) {
    uint4 v = rocrand4(&st);
    std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
