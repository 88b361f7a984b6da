// Host-only probe: prints rocRAND's Philox4x32-10 block for each
// "c0 c1 c2 c3 k0 k1" line read from stdin (library routine used as a pin).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Probe : rocrand_device::philox4x32_10_engine {
  uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  Probe p;
  unsigned a, b, c, d, e, f;
  while (std::scanf("%u %u %u %u %u %u", &a, &b, &c, &d, &e, &f) == 6) {
    uint4 ctr = {a, b, c, d};
    uint2 key = {e, f};
    uint4 o = p.run(ctr, key);
    std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
  }
  return 0;
}
