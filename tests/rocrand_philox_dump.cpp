// Prints Philox4x32-10 blocks from rocRAND's host-callable engine, used as an
// independent implementation to pin the oracle's generator. For each line of
// stdin "seed subsequence" it prints the four 32-bit words of the first block,
// i.e. the cipher of counter (0, 0, lo(subsequence), hi(subsequence)) under
// key (lo(seed), hi(seed)).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned long long seed, sub;
  while (std::scanf("%llu %llu", &seed, &sub) == 2) {
    rocrand_device::philox4x32_10_engine e(seed, sub, 0);
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
