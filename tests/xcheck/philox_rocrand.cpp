// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) and prints the four output words of
// Philox4x32-10 as computed by rocRAND's device header (host-compiled), an
// implementation independent of the oracle.  The protected ten-round block
// function is reached through a derived class.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdint>

struct Block : rocrand_device::philox4x32_10_engine {
  uint4 run(uint4 ctr, uint2 key) { return this->ten_rounds(ctr, key); }
};

int main() {
  unsigned int c0, c1, c2, c3, k0, k1;
  Block b;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 ctr; ctr.x = c0; ctr.y = c1; ctr.z = c2; ctr.w = c3;
    uint2 key; key.x = k0; key.y = k1;
    uint4 r = b.run(ctr, key);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
