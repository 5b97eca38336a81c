// lbl_device.hpp -- device-side building blocks of the gfx950 sweep:
// lattice tables, the orthonormal mode basis (built at compile time), the
// Philox4x32-10 counter generator with Box-Muller normals, and periodic
// indexing.  Everything here is header-only and constexpr where possible so
// that fully unrolled loops fold the tables into immediates.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "lbl_math.hpp"

namespace lbl {

constexpr double kCs2 = 1.0 / 3.0;  // c_s^2 for dx = dt = 1 (Sec. VI)

// ---------------------------------------------------------------------------
// Velocity sets in the canonical order of the C ABI.
// ---------------------------------------------------------------------------
template <int Q>
struct Lat;

template <>
struct Lat<9> {
  static constexpr int Q = 9, D = 2, NSTRESS = 3, NLINKS = 4;
  static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                  1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  // Monomials whose Gram-Schmidt orthonormalisation is the mode basis:
  // 1, x, y, x^2+y^2, x^2-y^2, xy, xy^2, x^2y, x^2y^2.
  static constexpr double mono(int k, double x, double y, double) {
    return k == 0 ? 1.0 : k == 1 ? x : k == 2 ? y : k == 3 ? x * x + y * y
         : k == 4 ? x * x - y * y : k == 5 ? x * y : k == 6 ? x * y * y
         : k == 7 ? x * x * y : x * x * y * y;
  }
  // Undirected Laplacian links (first non-zero component +1), by |c|^2 then
  // descending lexicographic order; weight 1/2 (|c|^2 = 1) or 1/4.
  static constexpr int lx[4] = {1, 0, 1, 1};
  static constexpr int ly[4] = {0, 1, 1, -1};
  static constexpr int lz[4] = {0, 0, 0, 0};
  static constexpr double lw[4] = {0.5, 0.5, 0.25, 0.25};
};

template <>
struct Lat<19> {
  static constexpr int Q = 19, D = 3, NSTRESS = 6, NLINKS = 13;
  static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                   1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  // 1, x, y, z, c^2, x^2, y^2, xy, xz, yz, xy^2, xz^2, yx^2, yz^2, zx^2, zy^2,
  // x^2y^2, x^2z^2, y^2z^2.
  static constexpr double mono(int k, double x, double y, double z) {
    return k == 0 ? 1.0 : k == 1 ? x : k == 2 ? y : k == 3 ? z
         : k == 4 ? x * x + y * y + z * z : k == 5 ? x * x : k == 6 ? y * y
         : k == 7 ? x * y : k == 8 ? x * z : k == 9 ? y * z
         : k == 10 ? x * y * y : k == 11 ? x * z * z : k == 12 ? y * x * x
         : k == 13 ? y * z * z : k == 14 ? z * x * x : k == 15 ? z * y * y
         : k == 16 ? x * x * y * y : k == 17 ? x * x * z * z : y * y * z * z;
  }
  // Shinozaki-Oono links: 6/22, 3/22, 1/22 by |c|^2 = 1, 2, 3.
  static constexpr int lx[13] = {1, 0, 0, 1, 1, 1, 1, 0, 0, 1, 1, 1, 1};
  static constexpr int ly[13] = {0, 1, 0, 1, 0, 0, -1, 1, 1, 1, 1, -1, -1};
  static constexpr int lz[13] = {0, 0, 1, 0, 1, -1, 0, 1, -1, 1, -1, 1, -1};
  static constexpr double lw[13] = {6.0 / 22, 6.0 / 22, 6.0 / 22, 3.0 / 22, 3.0 / 22,
                                    3.0 / 22, 3.0 / 22, 3.0 / 22, 3.0 / 22, 1.0 / 22,
                                    1.0 / 22, 1.0 / 22, 1.0 / 22};
};

// D3Q15, the paper's own lattice (Sec. VI): rest 2/9, axes 1/9, cube
// corners 1/72.
template <>
struct Lat<15> {
  static constexpr int Q = 15, D = 3, NSTRESS = 6, NLINKS = 13;
  static constexpr int cx[15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
  static constexpr int cy[15] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
  static constexpr int cz[15] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1};
  static constexpr double w[15] = {2.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,
                                   1.0 / 9,  1.0 / 9,  1.0 / 72, 1.0 / 72, 1.0 / 72,
                                   1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72};
  // 1, x, y, z, c^2, x^2, y^2, xy, xz, yz, x c^2, y c^2, z c^2, c^4, xyz.
  static constexpr double mono(int k, double x, double y, double z) {
    return k == 0 ? 1.0 : k == 1 ? x : k == 2 ? y : k == 3 ? z
         : k == 4 ? x * x + y * y + z * z : k == 5 ? x * x : k == 6 ? y * y
         : k == 7 ? x * y : k == 8 ? x * z : k == 9 ? y * z
         : k == 10 ? x * (x * x + y * y + z * z) : k == 11 ? y * (x * x + y * y + z * z)
         : k == 12 ? z * (x * x + y * y + z * z)
         : k == 13 ? (x * x + y * y + z * z) * (x * x + y * y + z * z) : x * y * z;
  }
  // The SMOL stencils do not depend on the LB lattice: Shinozaki-Oono links.
  static constexpr int lx[13] = {1, 0, 0, 1, 1, 1, 1, 0, 0, 1, 1, 1, 1};
  static constexpr int ly[13] = {0, 1, 0, 1, 0, 0, -1, 1, 1, 1, 1, -1, -1};
  static constexpr int lz[13] = {0, 0, 1, 0, 1, -1, 0, 1, -1, 1, -1, 1, -1};
  static constexpr double lw[13] = {6.0 / 22, 6.0 / 22, 6.0 / 22, 3.0 / 22, 3.0 / 22,
                                    3.0 / 22, 3.0 / 22, 3.0 / 22, 3.0 / 22, 1.0 / 22,
                                    1.0 / 22, 1.0 / 22, 1.0 / 22};
};

// ---------------------------------------------------------------------------
// Compile-time orthonormal mode basis: classical Gram-Schmidt of the
// monomials under <a,b> = sum_i w_i a(c_i) b(c_i).  e[k][i] = e_k(c_i).
// ---------------------------------------------------------------------------
constexpr double ce_sqrt(double x) {
  double r = x > 1.0 ? x : 1.0;
  for (int it = 0; it < 200; ++it) r = 0.5 * (r + x / r);
  return r;
}

template <int Q>
struct Basis {
  double e[Q][Q];
};

template <int Q>
constexpr Basis<Q> make_basis() {
  using L = Lat<Q>;
  Basis<Q> B{};
  for (int k = 0; k < Q; ++k) {
    double m[Q] = {};
    double v[Q] = {};
    for (int i = 0; i < Q; ++i) {
      m[i] = L::mono(k, L::cx[i], L::cy[i], L::cz[i]);
      v[i] = m[i];
    }
    for (int l = 0; l < k; ++l) {
      double pr = 0.0;
      for (int i = 0; i < Q; ++i) pr += L::w[i] * m[i] * B.e[l][i];
      for (int i = 0; i < Q; ++i) v[i] -= pr * B.e[l][i];
    }
    double n2 = 0.0;
    for (int i = 0; i < Q; ++i) n2 += L::w[i] * v[i] * v[i];
    double n = ce_sqrt(n2);
    for (int i = 0; i < Q; ++i) B.e[k][i] = v[i] / n;
  }
  return B;
}

template <int Q>
struct Modes {
  static constexpr Basis<Q> B = make_basis<Q>();
};

// Every basis vector is a scale times a vector of small integers:
// e_k(c_i) = scale[k] * I[k][i].  Kernels project with the integers (inline
// constants) and one multiply by the scale per mode.
template <int Q>
struct IntBasis {
  double scale[Q];
  int I[Q][Q];
};

constexpr double ce_abs(double v) { return v < 0 ? -v : v; }
constexpr int ce_round(double v) { return v >= 0 ? static_cast<int>(v + 0.5) : -static_cast<int>(-v + 0.5); }

template <int Q>
constexpr IntBasis<Q> make_int_basis() {
  const Basis<Q> B = make_basis<Q>();
  IntBasis<Q> R{};
  for (int k = 0; k < Q; ++k) {
    double mn = 1e300;
    for (int i = 0; i < Q; ++i)
      if (ce_abs(B.e[k][i]) > 1e-9 && ce_abs(B.e[k][i]) < mn) mn = ce_abs(B.e[k][i]);
    R.scale[k] = mn;
    for (int i = 0; i < Q; ++i) R.I[k][i] = ce_round(B.e[k][i] / mn);
  }
  return R;
}

template <int Q>
constexpr double int_basis_error() {
  const Basis<Q> B = make_basis<Q>();
  const IntBasis<Q> R = make_int_basis<Q>();
  double err = 0.0;
  for (int k = 0; k < Q; ++k)
    for (int i = 0; i < Q; ++i) {
      const double e = ce_abs(B.e[k][i] - R.scale[k] * R.I[k][i]);
      if (e > err) err = e;
    }
  return err;
}

template <int Q>
struct IntModes {
  static constexpr IntBasis<Q> B = make_int_basis<Q>();
  static_assert(int_basis_error<Q>() < 1e-13, "mode basis is not scale x integers");
};

// Entries as variable templates: always compile-time constants in kernels.
template <int Q, int K, int I>
inline constexpr int kIB = IntModes<Q>::B.I[K][I];
template <int Q, int K>
inline constexpr double kSB = IntModes<Q>::B.scale[K];

// Compile-time loop: f(std::integral_constant<int, 0>{}) ... f(<N-1>).
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// ---------------------------------------------------------------------------
struct u32x4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c.x;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c.z;
    c = u32x4{static_cast<uint32_t>(p1 >> 32) ^ c.y ^ k0, static_cast<uint32_t>(p1),
              static_cast<uint32_t>(p0 >> 32) ^ c.w ^ k1, static_cast<uint32_t>(p0)};
  }
  return c;
}

enum : uint32_t { kTagLB = 0, kTagSMOL = 1, kTagInit = 2 };

// Four normals of Philox block (site, step, block, tag): uniforms
// (x + 1/2) 2^-32, Box-Muller on (u0,u1) and (u2,u3).
template <typename C>
struct Normal4;

// Square root of a in [1e-10, 1e2] (the radii of Box-Muller, -2 ln u with
// u in [2^-33, 1 - 2^-33]): the hardware reciprocal square root refined by
// two coupled Newton (Goldschmidt) iterations for g ~ sqrt(a), h ~ 1/(2 sqrt a),
// then one residual correction g + (a - g^2) h.  No scaling or special cases
// are needed on this range.
__device__ __forceinline__ double sqrt_radius(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, a);
  return fma(d, h, g);
}

template <>
struct Normal4<double> {
  // Box-Muller pair from two 32-bit outputs: sqrt(-2 ln u_a) (cos, sin)(2 pi u_b).
  __device__ __forceinline__ static void pair(uint32_t ka, uint32_t kb, double& za, double& zb) {
    const double r = sqrt_radius(-2.0 * bm::log_unit(bm::unit(ka)));
    double s, c;
    bm::sincos_turn(kb, &s, &c);
    za = r * c;
    zb = r * s;
  }
  __device__ __forceinline__ static void gen(uint32_t site, uint32_t step, uint32_t block,
                                             uint32_t tag, uint32_t k0, uint32_t k1,
                                             double z[4]) {
    const u32x4 r = philox4x32_10(u32x4{site, step, block, tag}, k0, k1);
    pair(r.x, r.y, z[0], z[1]);
    pair(r.z, r.w, z[2], z[3]);
  }
  // Only the first pair (slots 0, 1 of the block).
  __device__ __forceinline__ static void gen2(uint32_t site, uint32_t step, uint32_t block,
                                              uint32_t tag, uint32_t k0, uint32_t k1,
                                              double z[2]) {
    const u32x4 r = philox4x32_10(u32x4{site, step, block, tag}, k0, k1);
    pair(r.x, r.y, z[0], z[1]);
  }
};

// FP32 storage: the transform in FP32 with the hardware transcendentals
// (log2, and sine and cosine of an angle given in turns, which is what the
// uniform already is).
template <>
struct Normal4<float> {
  __device__ __forceinline__ static float unif(uint32_t x) {
    return fmaf(static_cast<float>(x), 0x1p-32f, 0x1p-33f);
  }
  __device__ __forceinline__ static void pair(uint32_t ka, uint32_t kb, float& za, float& zb) {
    constexpr float kMinus2Ln2 = -1.38629436111989061883f;  // -2 ln 2
    const float r = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(unif(ka)));
    const float t = unif(kb);
    za = r * __builtin_amdgcn_cosf(t);
    zb = r * __builtin_amdgcn_sinf(t);
  }
  __device__ __forceinline__ static void gen(uint32_t site, uint32_t step, uint32_t block,
                                             uint32_t tag, uint32_t k0, uint32_t k1, float z[4]) {
    const u32x4 r = philox4x32_10(u32x4{site, step, block, tag}, k0, k1);
    pair(r.x, r.y, z[0], z[1]);
    pair(r.z, r.w, z[2], z[3]);
  }
  __device__ __forceinline__ static void gen2(uint32_t site, uint32_t step, uint32_t block,
                                              uint32_t tag, uint32_t k0, uint32_t k1,
                                              float z[2]) {
    const u32x4 r = philox4x32_10(u32x4{site, step, block, tag}, k0, k1);
    pair(r.x, r.y, z[0], z[1]);
  }
};

// Normal of one slot (used where only a single value of a block is needed).
template <typename C>
__device__ __forceinline__ C normal_slot(uint32_t site, uint32_t step, uint32_t slot,
                                         uint32_t tag, uint32_t k0, uint32_t k1) {
  C z[4];
  Normal4<C>::gen(site, step, slot >> 2, tag, k0, k1, z);
  const uint32_t lane = slot & 3u;
  return lane == 0 ? z[0] : lane == 1 ? z[1] : lane == 2 ? z[2] : z[3];
}

// ---------------------------------------------------------------------------
// Periodic lattice geometry.
// ---------------------------------------------------------------------------
struct Geom {
  int nx, ny, nz;
  int N;
  __device__ __forceinline__ int wrapx(int x) const { return x < 0 ? x + nx : (x >= nx ? x - nx : x); }
  __device__ __forceinline__ int wrapy(int y) const { return y < 0 ? y + ny : (y >= ny ? y - ny : y); }
  __device__ __forceinline__ int wrapz(int z) const { return z < 0 ? z + nz : (z >= nz ? z - nz : z); }
  __device__ __forceinline__ int idx(int x, int y, int z) const { return x + nx * (y + ny * z); }
  // Site at (x+dx, y+dy, z+dz) for |d| <= 1 per axis (lattice sides >= 4).
  __device__ __forceinline__ int nb(int x, int y, int z, int dx, int dy, int dz) const {
    return idx(wrapx(x + dx), wrapy(y + dy), wrapz(z + dz));
  }
};

}  // namespace lbl
