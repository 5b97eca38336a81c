// lbl_math.hpp -- the elementary functions of the Box-Muller transform,
// specialised to the only arguments it ever sees: uniforms u = (k + 1/2) 2^-32
// with k a 32-bit Philox output.  Knowing the argument set lets the range
// reduction happen exactly (in the exponent field for the logarithm, in the
// integer k for the angle), so only short polynomials remain.  Accuracy is a
// few units in the last place of FP64 over the whole set, which keeps the
// normals within rounding of any correctly rounded libm evaluation.
//
// The functions are __host__ __device__ so that the same code can be checked
// against extended-precision references on the host.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

namespace lbl {
namespace bm {

// u = (k + 1/2) 2^-32, exact in FP64.
__host__ __device__ inline double unit(uint32_t k) {
  return (static_cast<double>(k) + 0.5) * 0x1p-32;
}

// ln u for u in (0, 1).  Write u = 2^e f with f in [sqrt(1/2), sqrt(2)), read
// off the exponent field; then ln f = 2 atanh(s) with s = (f - 1)/(f + 1),
// |s| <= 3 - 2 sqrt(2), summed as s * sum_k 2 s^{2k} / (2k + 1) up to k = 10
// (truncation below 1e-18 relative).  f - 1 is exact, so u close to 1 keeps
// its full relative accuracy.
__host__ __device__ inline double log_unit(double u) {
  uint64_t bits;
  memcpy(&bits, &u, sizeof bits);
  int e = static_cast<int>((bits >> 52) & 0x7ff) - 1022;  // u = f 2^e, f in [1/2, 1)
  bits = (bits & 0x000fffffffffffffULL) | (0x3feULL << 52);
  double f;
  memcpy(&f, &bits, sizeof f);
  if (f < 0.70710678118654752440) {
    f *= 2.0;
    e -= 1;
  }
  const double s = (f - 1.0) / (f + 1.0);
  const double z = s * s;
  double p = 2.0 / 21.0;
  p = fma(z, p, 2.0 / 19.0);
  p = fma(z, p, 2.0 / 17.0);
  p = fma(z, p, 2.0 / 15.0);
  p = fma(z, p, 2.0 / 13.0);
  p = fma(z, p, 2.0 / 11.0);
  p = fma(z, p, 2.0 / 9.0);
  p = fma(z, p, 2.0 / 7.0);
  p = fma(z, p, 2.0 / 5.0);
  p = fma(z, p, 2.0 / 3.0);
  // ln f = 2 s + s z p; ln 2 split so that e * kLn2Hi is exact (|e| <= 34).
  constexpr double kLn2Hi = 0x1.62e42fefa3800p-1, kLn2Lo = 0x1.ef35793c76730p-45;
  const double de = static_cast<double>(e);
  const double lnf = fma(s * z, p, 2.0 * s);
  return fma(de, kLn2Hi, fma(de, kLn2Lo, lnf));
}

// sin and cos of phi in [0, pi/4] by their Taylor series (through phi^15 and
// phi^16; truncation below 1e-17).
__host__ __device__ inline void sincos_octant(double phi, double* s, double* c) {
  const double z = phi * phi;
  double ps = -1.0 / 1307674368000.0;  // -1/15!
  ps = fma(z, ps, 1.0 / 6227020800.0);  // 1/13!
  ps = fma(z, ps, -1.0 / 39916800.0);   // -1/11!
  ps = fma(z, ps, 1.0 / 362880.0);      // 1/9!
  ps = fma(z, ps, -1.0 / 5040.0);       // -1/7!
  ps = fma(z, ps, 1.0 / 120.0);         // 1/5!
  ps = fma(z, ps, -1.0 / 6.0);          // -1/3!
  *s = fma(phi * z, ps, phi);
  double pc = 1.0 / 20922789888000.0;   // 1/16!
  pc = fma(z, pc, -1.0 / 87178291200.0);  // -1/14!
  pc = fma(z, pc, 1.0 / 479001600.0);     // 1/12!
  pc = fma(z, pc, -1.0 / 3628800.0);      // -1/10!
  pc = fma(z, pc, 1.0 / 40320.0);         // 1/8!
  pc = fma(z, pc, -1.0 / 720.0);          // -1/6!
  pc = fma(z, pc, 1.0 / 24.0);            // 1/4!
  pc = fma(z, pc, -0.5);
  *c = fma(z, pc, 1.0);
}

// sin and cos of 2 pi u with u = (k + 1/2) 2^-32.  The top two bits of k give
// the quadrant; within it, an angle past pi/4 is reflected to pi/2 minus it
// (exactly, on the integer: (2^30 - 1 - r) + 1/2 = 2^30 - (r + 1/2)), which
// swaps sine and cosine.
__host__ __device__ inline void sincos_turn(uint32_t k, double* s, double* c) {
  const uint32_t quad = k >> 30;
  uint32_t r = k & 0x3fffffffu;
  const bool refl = (r >> 29) != 0;
  if (refl) r = 0x3fffffffu - r;
  constexpr double kTurn = 0x1.921fb54442d18p-30;  // 2 pi 2^-32
  const double phi = (static_cast<double>(r) + 0.5) * kTurn;
  double sp, cp;
  sincos_octant(phi, &sp, &cp);
  // The reflection swaps sine and cosine, and so does a rotation by an odd
  // multiple of pi/2: one swap for both.  Then the signs of the rotation by
  // quad * pi/2: sine negative in quadrants 2, 3, cosine in 1, 2.
  const bool swap = refl != ((quad & 1u) != 0);
  const double so = swap ? cp : sp;
  const double co = swap ? sp : cp;
  *s = (quad & 2u) ? -so : so;
  *c = ((quad + 1u) & 2u) ? -co : co;
}

}  // namespace bm
}  // namespace lbl
