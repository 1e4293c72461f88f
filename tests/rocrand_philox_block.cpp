// Host-side Philox4x32-10 block function of rocRAND (its device header
// compiled for the host), used by the CPU tests as a library reference for
// the oracle's own implementation.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal
// 32-bit words, c0 the lowest counter word) and prints the four output words.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

namespace {
struct Block : rocrand_device::philox4x32_10_engine {
  uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
}  // namespace

int main() {
  Block b;
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    const uint4 r = b.run(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
