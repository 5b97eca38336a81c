// Host check of the Box-Muller elementary functions of the GPU sweep against
// extended-precision libm: prints the worst errors in units of 2^-52 (relative
// for the logarithm, absolute for sine and cosine, whose values are <= 1).
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstdint>

#include "lbl_math.hpp"

static uint64_t lcg = 0x9e3779b97f4a7c15ULL;
static uint32_t next_u32() {
  lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
  return static_cast<uint32_t>(lcg >> 32);
}

int main(int argc, char** argv) {
  const long n = argc > 1 ? std::atol(argv[1]) : 2000000;
  const long double two_pi = 6.283185307179586476925286766559005768L;
  double worst_log = 0, worst_sin = 0, worst_cos = 0, worst_pyth = 0;
  uint32_t at_log = 0, at_sin = 0, at_cos = 0;
  const uint32_t edges[] = {0u, 1u, 2u, 3u, 0x1fffffffu, 0x20000000u, 0x3fffffffu, 0x40000000u,
                            0x5fffffffu, 0x60000000u, 0x7fffffffu, 0x80000000u, 0x9fffffffu,
                            0xa0000000u, 0xbfffffffu, 0xc0000000u, 0xdfffffffu, 0xe0000000u,
                            0xfffffffeu, 0xffffffffu, 0xb504f333u, 0xb504f334u, 0x6a09e667u};
  const long ne = sizeof(edges) / sizeof(edges[0]);
  for (long i = 0; i < n + ne; ++i) {
    const uint32_t k = i < ne ? edges[i] : next_u32();
    const double u = lbl::bm::unit(k);
    const long double ul = (static_cast<long double>(k) + 0.5L) / 4294967296.0L;
    const long double lref = logl(ul);
    const double lg = lbl::bm::log_unit(u);
    const double el = static_cast<double>(fabsl((lg - lref) / lref)) / 0x1p-52;
    if (el > worst_log) { worst_log = el; at_log = k; }
    double s, c;
    lbl::bm::sincos_turn(k, &s, &c);
    const long double ang = two_pi * ul;
    const double es = static_cast<double>(fabsl(s - sinl(ang))) / 0x1p-52;
    const double ec = static_cast<double>(fabsl(c - cosl(ang))) / 0x1p-52;
    if (es > worst_sin) { worst_sin = es; at_sin = k; }
    if (ec > worst_cos) { worst_cos = ec; at_cos = k; }
    const double ep = std::fabs(s * s + c * c - 1.0) / 0x1p-52;
    if (ep > worst_pyth) worst_pyth = ep;
  }
  std::printf("log_rel_ulp %.3f at %u\nsin_abs_ulp %.3f at %u\ncos_abs_ulp %.3f at %u\npyth_ulp %.3f\n",
              worst_log, at_log, worst_sin, at_sin, worst_cos, at_cos, worst_pyth);
  return 0;
}
