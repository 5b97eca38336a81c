// Host-side reference for the oracle's Philox4x32-10: evaluates rocRAND's
// independent implementation (its header-only engine) on counters and keys
// read from stdin, one "c0 c1 c2 c3 k0 k1" hexadecimal line per query.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

struct philox_probe : rocrand_device::philox4x32_10_engine {
  uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
  philox_probe p;
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = p.rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
