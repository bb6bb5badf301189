// Host-side driver for rocRAND's Philox4x32-10 bijection (its header's
// ten_rounds function, compiled for the CPU).  Used only by the test that
// pins the oracle's generator to an independent library implementation.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) on stdin, writes the four
// output words per line.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

// ten_rounds is a protected member of the engine; a derived class exposes it.
struct philox_bijection : rocrand_device::philox4x32_10_engine {
  uint4 apply(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};

int main() {
  philox_bijection eng;
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 ctr{c0, c1, c2, c3};
    uint2 key{k0, k1};
    uint4 r = eng.apply(ctr, key);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
