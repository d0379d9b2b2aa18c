// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) and prints the four output words of
// Philox4x32-10 as computed by ATen's PhiloxRNGEngine.h (an implementation of
// the SC'11 generator that is independent of the oracle).  The counter is set
// through the public API: key = seed, (c2, c3) = subsequence, (c0, c1) = offset.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    uint64_t subseq = (uint64_t)c2 | ((uint64_t)c3 << 32);
    at::philox_engine eng(seed, subseq, 0);
    eng.set_offset((uint64_t)c0 | ((uint64_t)c1 << 32));
    uint32_t r0 = eng(), r1 = eng(), r2 = eng(), r3 = eng();
    std::printf("%u %u %u %u\n", r0, r1, r2, r3);
  }
  return 0;
}
