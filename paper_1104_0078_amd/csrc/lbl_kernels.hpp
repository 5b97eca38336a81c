// lbl_kernels.hpp -- gfx950 kernels of the coupled FLBE + SMOL step.
//
// Storage type S is double (FP64 path) or float (FP32-deviation path, where
// populations hold fbar_i - w_i rho0).  Arithmetic runs in S.
//
// Per step (full coupling), in launch order:
//   k_prep_*    mu(psi^n) for the LB force and the SMOL noise N^n (frozen
//               over the stages); z-marching tiles, noise folded through LDS
//   k_lb        pull-stream, force -psi grad mu, MRT collision with noise,
//               writes f*^n and u^n                          one thread/site
//   k_lb (no collision, "k_uend")  velocity of the streamed populations,
//               (jbar^{n+1} + F^n/2)/rho^{n+1}, for the stages at t_{n+1}
//   k_stage_*   one Runge-Kutta stage: phi -> mu(phi) -> fluxes -> divergence
//               (z-marching tiles, per-plane stencil sums carried in
//               registers); once per stage
// Options: the FD noise built in Fourier space (k_white, a hipFFT pair,
// k_fourier_scale) in place of the link fluxes of k_prep_fd; the force as the
// divergence of the order-parameter stress (k_stress, k_force_stress; for FV
// in 3-D the single z-marching pass k_stress_force_fv3), read by k_lb in
// place of -psi grad mu.  k_mu (mu alone) serves the velocity
// observable.  Populations are structure-of-arrays f[i*N + s]; the stored
// buffer holds the post-collision values f*^{n-1} and step n pulls
// fbar^n(x) = f*^{n-1}(x - c_i).
#pragma once

#include "lbl_device.hpp"

namespace lbl {

enum : int { kFD = 0, kFV = 1 };

template <typename S>
struct Coef {
  S a, b, kappa, M;
};

// Thread-block shape of the batched per-site kernels: 64 sites along x (one
// wavefront, contiguous in memory) by 4 rows.
constexpr int kBX = 64, kBY = 4;
constexpr int kSiteBlock = 256;  // threads per block of the per-site kernels
// Tile of the z-marching stencil kernels.
constexpr int kTX = 32, kTY = 8;

// Schedule of the single-simulation per-site kernels: 256-thread blocks that
// cover 2^lw sites along x by 256 / 2^lw rows of one z-plane, enumerated with
// x fastest.  The hardware hands the blocks of a 1-D grid to the 8 XCDs
// round-robin; with `per` > 0 block b takes virtual block (b % 8) per + b / 8,
// so each XCD sweeps one contiguous eighth of the lattice and the rows that a
// pull reads across block edges sit in the same L2.
struct SiteMap {
  int lw;        // log2 of the block width along x
  int nbx, nby;  // blocks along x and y
  int nb;        // blocks in total
  int per;       // blocks per XCD when swizzled, else 0
};

__host__ inline SiteMap make_site_map(int nx, int ny, int nz, int lw, bool swizzle) {
  SiteMap m;
  m.lw = lw;
  const int w = 1 << lw, h = kSiteBlock >> lw;
  m.nbx = (nx + w - 1) / w;
  m.nby = (ny + h - 1) / h;
  m.nb = m.nbx * m.nby * nz;
  m.per = swizzle ? (m.nb + 7) / 8 : 0;
  return m;
}

__host__ inline int site_map_blocks(const SiteMap& m) { return m.per ? 8 * m.per : m.nb; }

// Site of this thread; false when the block is padding or the site is off
// the lattice.
__device__ __forceinline__ bool site_of(const SiteMap& m, const Geom& g, int& x, int& y, int& z) {
  int b = blockIdx.x;
  if (m.per) {
    b = (b & 7) * m.per + (b >> 3);
    if (b >= m.nb) return false;
  }
  const int bx = b % m.nbx, r = b / m.nbx;
  const int by = r % m.nby;
  z = r / m.nby;
  x = (bx << m.lw) + (threadIdx.x & ((1 << m.lw) - 1));
  y = by * (kSiteBlock >> m.lw) + (threadIdx.x >> m.lw);
  return x < g.nx && y < g.ny;
}

// Schedule of the single-simulation z-marching tile kernels: a 1-D grid over
// ntx x nty x nzc tiles (x fastest); with `per` > 0 block b takes virtual tile
// (b % 8) per + b / 8, so each XCD marches a contiguous range of tiles and the
// halo rows that neighbouring tiles re-read stay in its L2.
struct TileMap {
  int ntx, nty;  // tiles along x and y
  int nt;        // tiles in total
  int per;       // tiles per XCD when swizzled, else 0
};

__host__ inline TileMap make_tile_map(int nx, int ny, int nzc, bool swizzle) {
  TileMap m;
  m.ntx = (nx + kTX - 1) / kTX;
  m.nty = (ny + kTY - 1) / kTY;
  m.nt = m.ntx * m.nty * nzc;
  m.per = swizzle ? (m.nt + 7) / 8 : 0;
  return m;
}

__host__ inline int tile_map_blocks(const TileMap& m) { return m.per ? 8 * m.per : m.nt; }

// Tile of this block; false for padding blocks.
__device__ __forceinline__ bool tile_of(const TileMap& m, int& bx, int& by, int& bz) {
  int b = blockIdx.x;
  if (m.per) {
    b = (b & 7) * m.per + (b >> 3);
    if (b >= m.nt) return false;
  }
  bx = b % m.ntx;
  const int r = b / m.ntx;
  by = r % m.nty;
  bz = r / m.nty;
  return true;
}

// Periodic neighbourhood of one site: wrapped coordinates and row offsets.
struct Nbr {
  int xs[3];
  int rows[3][3];  // rows[dy+1][dz+1] = nx * (y+dy + ny * (z+dz))
  __device__ __forceinline__ Nbr(const Geom& g, int x, int y, int z) {
    xs[0] = x == 0 ? g.nx - 1 : x - 1;
    xs[1] = x;
    xs[2] = x == g.nx - 1 ? 0 : x + 1;
    const int ys[3] = {y == 0 ? g.ny - 1 : y - 1, y, y == g.ny - 1 ? 0 : y + 1};
    const int zs[3] = {z == 0 ? g.nz - 1 : z - 1, z, z == g.nz - 1 ? 0 : z + 1};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int zr = g.ny * zs[b];
#pragma unroll
      for (int a = 0; a < 3; ++a) rows[a][b] = g.nx * (ys[a] + zr);
    }
  }
  __device__ __forceinline__ int at(int dx, int dy, int dz) const {
    return xs[dx + 1] + rows[dy + 1][dz + 1];
  }
};

__device__ __forceinline__ int wrap_any(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Periodic wrap of a tile-region coordinate v in [-halo, start + tile + halo):
// one conditional add or subtract when the side n is at least tile + halo
// (`near`, uniform per launch), a modulo otherwise.
__device__ __forceinline__ int wrap_r(int v, int n, bool near) {
  if (near) return v < 0 ? v + n : (v >= n ? v - n : v);
  return wrap_any(v, n);
}

// ---------------------------------------------------------------------------
// Chemical potential mu = A phi + B phi^3 - K L_SO phi  (Sec. II.A; the
// Shinozaki-Oono Laplacian of Eq. (solap) in 3-D, its 2-D analogue in 2-D).
// `at(dx,dy,dz)` returns phi at the offset.
// ---------------------------------------------------------------------------
template <typename S, int D, class At>
__device__ __forceinline__ S lap_so(At&& at) {
  S s1 = 0, s2 = 0, s3 = 0;
  if constexpr (D == 3) {
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int r2 = dx * dx + dy * dy + dz * dz;
          if (r2 == 0) continue;
          const S v = at(dx, dy, dz);
          if (r2 == 1) s1 += v;
          else if (r2 == 2) s2 += v;
          else s3 += v;
        }
    return S(6.0 / 22.0) * s1 + S(3.0 / 22.0) * s2 + S(1.0 / 22.0) * s3 -
           S(80.0 / 22.0) * at(0, 0, 0);
  } else {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int r2 = dx * dx + dy * dy;
        if (r2 == 0) continue;
        const S v = at(dx, dy, 0);
        if (r2 == 1) s1 += v;
        else s2 += v;
      }
    return S(0.5) * s1 + S(0.25) * s2 - S(3.0) * at(0, 0, 0);
  }
}

template <typename S, int D, class At>
__device__ __forceinline__ S chem_pot(const Coef<S>& c, At&& at) {
  const S p = at(0, 0, 0);
  return c.a * p + c.b * p * p * p - c.kappa * lap_so<S, D>(at);
}

// The 3-D Shinozaki-Oono Laplacian split by planes for z-marching kernels: with
// the centre value c, the 4-face sum f and the 4-corner sum k of each plane,
// L_SO phi = (6 F + 3 E + C - 80 phi)/22 where F = f_z + c_{z-1} + c_{z+1},
// E = k_z + f_{z-1} + f_{z+1}, C = k_{z-1} + k_{z+1} (face, edge and corner
// neighbours).  A thread pushes the sums of each new plane (9 LDS reads) and
// evaluates mu at the middle one of the last three, instead of 27 reads.
template <typename S>
struct SoPlanes {
  S c[3], f[3], k[3];  // planes z-1, z, z+1 (slot 2 newest)
  __device__ __forceinline__ SoPlanes() {
#pragma unroll
    for (int r = 0; r < 3; ++r) c[r] = f[r] = k[r] = S(0);
  }
  // P points at the centre of the new plane in an LDS row layout of width W.
  template <int W>
  __device__ __forceinline__ void push(const S* P) {
    c[2] = P[0];
    f[2] = (P[-1] + P[1]) + (P[-W] + P[W]);
    k[2] = (P[-W - 1] + P[-W + 1]) + (P[W - 1] + P[W + 1]);
  }
  // L_SO phi at the middle plane.
  __device__ __forceinline__ S lap() const {
    const S F = f[1] + (c[0] + c[2]);
    const S E = k[1] + (f[0] + f[2]);
    const S C = k[0] + k[2];
    return S(6.0 / 22.0) * F + S(3.0 / 22.0) * E + S(1.0 / 22.0) * C - S(80.0 / 22.0) * c[1];
  }
  __device__ __forceinline__ S mu(const Coef<S>& co) const {
    const S ph = c[1];
    const S lp = lap();
    return co.a * ph + co.b * ph * ph * ph - co.kappa * lp;
  }
  __device__ __forceinline__ void roll() {
    c[0] = c[1];
    c[1] = c[2];
    f[0] = f[1];
    f[1] = f[2];
    k[0] = k[1];
    k[1] = k[2];
  }
  // mu at the middle plane with the plane below (lo) or above (hi) beyond a
  // wall: every link into it takes the centre value, i.e. that plane reads
  // as uniform at c[1] (centre, 4 faces, 4 corners).
  __device__ __forceinline__ S mu_walled(const Coef<S>& co, bool lo, bool hi) const {
    SoPlanes<S> w = *this;
    if (lo) {
      w.c[0] = c[1];
      w.f[0] = S(4) * c[1];
      w.k[0] = S(4) * c[1];
    }
    if (hi) {
      w.c[2] = c[1];
      w.f[2] = S(4) * c[1];
      w.k[2] = S(4) * c[1];
    }
    return w.mu(co);
  }
};

template <typename S, int Q>
__global__ __launch_bounds__(kBX* kBY) void k_mu(Geom g, Coef<S> c, const S* __restrict__ phi,
                                                 S* __restrict__ mu) {
  const int x = blockIdx.x * kBX + threadIdx.x, y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const Nbr nb(g, x, y, z);
  mu[nb.at(0, 0, 0)] =
      chem_pot<S, Lat<Q>::D>(c, [&](int dx, int dy, int dz) { return phi[nb.at(dx, dy, dz)]; });
}

// ---------------------------------------------------------------------------
// Force as the divergence of the order-parameter stress (Eq. muf):
//   sigma_ab = K g_a g_b + delta_ab [A psi^2/2 + 3 B psi^4/4 - K psi L psi - K/2 |g|^2],
//   F_a = -sum_b G_b sigma_ab,
// with g = G psi, G the variant's gradient (FD: central difference; FV:
// (1/c_s^2) sum_i w_i c_i (.)(x + c_i)) and L the Shinozaki-Oono Laplacian.
// Every term of F is a difference of shifted copies, so the sum of F over the
// lattice vanishes for any B.  sigma is stored by its d(d+1)/2 independent
// components: xx, yy, (zz,) xy(, xz, yz).
// ---------------------------------------------------------------------------
template <int D>
__host__ __device__ constexpr int sym_idx(int a, int b) {
  return a == b ? a : (D == 2 ? 2 : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5)));
}

template <typename S, int Q, int SMOL>
__device__ __forceinline__ void grad_at(const Nbr& nb, const S* __restrict__ v, S (&gr)[3]) {
  using L = Lat<Q>;
  gr[0] = gr[1] = gr[2] = S(0);
  if constexpr (SMOL == kFD) {
    gr[0] = S(0.5) * (v[nb.at(1, 0, 0)] - v[nb.at(-1, 0, 0)]);
    gr[1] = S(0.5) * (v[nb.at(0, 1, 0)] - v[nb.at(0, -1, 0)]);
    if (L::D == 3) gr[2] = S(0.5) * (v[nb.at(0, 0, 1)] - v[nb.at(0, 0, -1)]);
  } else {
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const S t = S(L::w[i]) * v[nb.at(L::cx[i], L::cy[i], L::cz[i])];
      if (L::cx[i]) gr[0] += L::cx[i] * t;
      if (L::cy[i]) gr[1] += L::cy[i] * t;
      if (L::cz[i]) gr[2] += L::cz[i] * t;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) gr[a] *= S(3);
  }
}

template <typename S, int Q, int SMOL>
__global__ __launch_bounds__(kBX* kBY) void k_stress(Geom g, Coef<S> c, const S* __restrict__ psi,
                                                     S* __restrict__ sig) {
  constexpr int D = Lat<Q>::D;
  const int x = blockIdx.x * kBX + threadIdx.x, y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const Nbr nb(g, x, y, z);
  const int s = nb.at(0, 0, 0);
  S gr[3];
  grad_at<S, Q, SMOL>(nb, psi, gr);
  const S ps = psi[s];
  const S lap = lap_so<S, D>([&](int dx, int dy, int dz) { return psi[nb.at(dx, dy, dz)]; });
  const S g2 = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
  const S iso = S(0.5) * c.a * ps * ps + S(0.75) * c.b * ps * ps * ps * ps - c.kappa * ps * lap -
                S(0.5) * c.kappa * g2;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = a; b < D; ++b)
      sig[static_cast<size_t>(sym_idx<D>(a, b)) * g.N + s] =
          c.kappa * gr[a] * gr[b] + (a == b ? iso : S(0));
}

template <typename S, int Q, int SMOL>
__global__ __launch_bounds__(kBX* kBY) void k_force_stress(Geom g, const S* __restrict__ sig,
                                                           S* __restrict__ F) {
  using L = Lat<Q>;
  constexpr int D = L::D, NS = D * (D + 1) / 2;
  const int x = blockIdx.x * kBX + threadIdx.x, y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const Nbr nb(g, x, y, z);
  S f[3] = {0, 0, 0};
  auto comp = [&](int k, int site) { return sig[static_cast<size_t>(k) * g.N + site]; };
  if constexpr (SMOL == kFD) {
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const int p = nb.at(b == 0, b == 1, b == 2), m = nb.at(-(b == 0), -(b == 1), -(b == 2));
#pragma unroll
      for (int a = 0; a < D; ++a)
        f[a] -= S(0.5) * (comp(sym_idx<D>(a, b), p) - comp(sym_idx<D>(a, b), m));
    }
  } else {
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int site = nb.at(L::cx[i], L::cy[i], L::cz[i]);
      S sv[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) sv[k] = comp(k, site);
      const int ci[3] = {L::cx[i], L::cy[i], L::cz[i]};
#pragma unroll
      for (int a = 0; a < D; ++a) {
        S acc = 0;
#pragma unroll
        for (int b = 0; b < D; ++b)
          if (ci[b]) acc += ci[b] * sv[sym_idx<D>(a, b)];
        f[a] -= S(3) * S(L::w[i]) * acc;
      }
    }
  }
  const int s = nb.at(0, 0, 0);
#pragma unroll
  for (int a = 0; a < D; ++a) F[static_cast<size_t>(a) * g.N + s] = f[a];
}

// ---------------------------------------------------------------------------
// FLBE: pull, moments, force, MRT collision with noise (App. B).
// ---------------------------------------------------------------------------
template <typename S>
struct LBArgs {
  Geom g;
  const S* f_in;  // f*^{n-1}
  S* f_out;       // f*^n
  const S* psi;   // psi^n
  const S* mu;    // mu(psi^n)
  S* u_out;       // u^n (d*N) or nullptr
  S rho0;
  S gamma_s, gamma_b, gamma_g;
  S sigma_s, sigma_b, sigma_g;
  uint32_t k0, k1, step;
  int force;  // 0: F = 0 (LB_ONLY)
  const S* Fext;  // force density given per site (d*N), else computed from mu
  int noise;  // 0: kT == 0
  int nt;     // host's choice of the NT kernel variant (see kStreamBytes)
  S uw[2][3];  // walls (WALLS kernels): velocities of the lower and upper wall
};

// Walls across the last axis (z in 3-D, y in 2-D), half a spacing below the
// first and above the last layer (the closing remark of Sec. V.B).  A pull
// from beyond a wall is a halfway bounce-back: the site's own reversed
// post-collision population plus Ladd's term 2 w_i rho0 c_i.U / c_s^2 of a
// wall moving at U.  In the stencils every link that crosses a wall is
// removed: a scalar field takes the centre's value beyond the wall, a flux
// field minus the centre's value.
template <int Q>
struct Opposite {
  int i[Q];
};

template <int Q>
constexpr Opposite<Q> make_opposite() {
  Opposite<Q> o{};
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j)
      if (Lat<Q>::cx[j] == -Lat<Q>::cx[i] && Lat<Q>::cy[j] == -Lat<Q>::cy[i] &&
          Lat<Q>::cz[j] == -Lat<Q>::cz[i])
        o.i[i] = j;
  return o;
}

template <int Q>
inline constexpr Opposite<Q> kOpp = make_opposite<Q>();

// Component of velocity i along the last axis.
template <int Q>
__host__ __device__ constexpr int c_last(int i) {
  return Lat<Q>::D == 3 ? Lat<Q>::cz[i] : Lat<Q>::cy[i];
}

// Weight sum of the velocities that cross one wall (c_last = +1; the same
// for -1 by symmetry): 1/6 on D3Q19 and D3Q15.  The flux rule of a wall
// (minus the centre's value beyond it) turns the links across it into
// -(sum of w_i c_i over them) . X(x) = +-W X_last(x).
template <int Q>
constexpr double wall_weight() {
  double s = 0;
  for (int i = 0; i < Q; ++i)
    if (c_last<Q>(i) > 0) s += Lat<Q>::w[i];
  return s;
}

// True when the offset (dy, dz) from a site at (y, z) leaves the lattice
// across a wall (D-dimensional lattice).
template <int D>
__device__ __forceinline__ bool beyond_wall(const Geom& g, int y, int z, int dy, int dz) {
  if constexpr (D == 3) {
    const int h = z + dz;
    return h < 0 || h >= g.nz;
  } else {
    const int h = y + dy;
    return h < 0 || h >= g.ny;
  }
}

// Launches whose populations outgrow the memory-side cache (256 MB on
// MI355X) stream them non-temporally; smaller working sets keep them cached.
constexpr double kStreamBytes = 256.0 * 1024 * 1024;

// GHOST: the ghost modes keep gamma_g m_g (omega_ghost != 1).
// COLLIDE: false computes only u (observable).
// WALLS: walls across the last axis (bounce-back pulls, one-sided force
// gradient next to a wall).
// The caller passes a site on the lattice.
template <typename S, bool DEV, int Q, int SMOL, bool GHOST, bool COLLIDE, bool NT,
          bool WALLS = false>
__device__ __forceinline__ void lb_body(const LBArgs<S>& a, int x, int y, int z) {
  using L = Lat<Q>;
  constexpr int D = L::D;
  constexpr int NR = Q - D - 1;
  constexpr int NB = (NR + 3) / 4;
  const Geom& g = a.g;
  const Nbr nb(g, x, y, z);
  const int s = nb.at(0, 0, 0);

  // The Q pulls go out first, the gathers of mu for the force behind them.
  S fv[Q];
  bool wlo = false, whi = false;
  if constexpr (WALLS) {
    const int h = D == 3 ? z : y, Lh = D == 3 ? g.nz : g.ny;
    wlo = h == 0;
    whi = h == Lh - 1;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const S* src = &a.f_in[static_cast<size_t>(i) * g.N + nb.at(-L::cx[i], -L::cy[i], -L::cz[i])];
    if constexpr (WALLS) {
      // the source lies beyond the lower (c_last > 0) or upper wall
      if ((c_last<Q>(i) > 0 && wlo) || (c_last<Q>(i) < 0 && whi)) {
        const S* U = c_last<Q>(i) > 0 ? a.uw[0] : a.uw[1];
        S cU = 0;
        if (L::cx[i]) cU += L::cx[i] * U[0];
        if (L::cy[i]) cU += L::cy[i] * U[1];
        if (L::cz[i]) cU += L::cz[i] * U[2];
        // one explicit fma: the same rounding in every kernel that inlines
        // this (the product is loop-invariant in the z-marching ones)
        fv[i] = fma(S(6.0 * L::w[i]) * a.rho0, cU,
                    a.f_in[static_cast<size_t>(kOpp<Q>.i[i]) * g.N + s]);
        continue;
      }
    }
    if constexpr (NT)
      fv[i] = __builtin_nontemporal_load(src);
    else
      fv[i] = *src;
  }

  // Force density F = -psi grad mu: FD central difference (Sec. IV) or the FV
  // gradient (1/c_s^2) sum_i w_i c_i mu(x + c_i) (Eq. fvgrad).
  S F[3] = {0, 0, 0};
  if (a.Fext) {
#pragma unroll
    for (int c = 0; c < D; ++c) F[c] = a.Fext[static_cast<size_t>(c) * g.N + s];
  } else if (a.force) {
    const S* __restrict__ mu = a.mu;
    S gx = 0, gy = 0, gz = 0;
    if constexpr (SMOL == kFD) {
      gx = S(0.5) * (mu[nb.at(1, 0, 0)] - mu[nb.at(-1, 0, 0)]);
      gy = S(0.5) * (mu[nb.at(0, 1, 0)] - mu[nb.at(0, -1, 0)]);
      if (D == 3) gz = S(0.5) * (mu[nb.at(0, 0, 1)] - mu[nb.at(0, 0, -1)]);
    } else {
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        int site = nb.at(L::cx[i], L::cy[i], L::cz[i]);
        if constexpr (WALLS)
          if (beyond_wall<D>(g, y, z, L::cy[i], L::cz[i])) site = s;
        const S t = S(L::w[i]) * mu[site];
        if (L::cx[i]) gx += L::cx[i] * t;
        if (L::cy[i]) gy += L::cy[i] * t;
        if (L::cz[i]) gz += L::cz[i] * t;
      }
      gx *= S(3);
      gy *= S(3);
      gz *= S(3);
    }
    const S ps = a.psi[s];
    F[0] = -ps * gx;
    F[1] = -ps * gy;
    F[2] = -ps * gz;
  }

  // Noise of the non-conserved modes, n_k = sigma_k z_k, with
  // sigma_k^2 = (1 - gamma_k^2) rho0 kT / c_s^2 per mode class.  Drawn after
  // the pulls are issued, so that its arithmetic overlaps their latency.
  S nk[NB * 4];
#pragma unroll
  for (int k = 0; k < NB * 4; ++k) nk[k] = 0;
  if (COLLIDE && a.noise) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      S z4[4];
      Normal4<S>::gen(static_cast<uint32_t>(s), a.step, b, kTagLB, a.k0, a.k1, z4);
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const int k = 4 * b + l;
        if (k >= NR) continue;
        const S sig = k == 0 ? a.sigma_b : (k < L::NSTRESS ? a.sigma_s : a.sigma_g);
        nk[k] = sig * z4[l];
      }
    }
  }

  S S0 = 0, jx = 0, jy = 0, jz = 0, pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const S v = fv[i];
    S0 += v;
    if (L::cx[i]) jx += L::cx[i] * v;
    if (L::cy[i]) jy += L::cy[i] * v;
    if (L::cz[i]) jz += L::cz[i] * v;
    if (L::cx[i]) pxx += v;
    if (L::cy[i]) pyy += v;
    if (L::cz[i]) pzz += v;
    if (L::cx[i] * L::cy[i]) pxy += (L::cx[i] * L::cy[i]) * v;
    if (L::cx[i] * L::cz[i]) pxz += (L::cx[i] * L::cz[i]) * v;
    if (L::cy[i] * L::cz[i]) pyz += (L::cy[i] * L::cz[i]) * v;
  }
  const S rho = DEV ? a.rho0 + S0 : S0;
  const S inv_rho = S(1) / rho;
  const S ux = (jx + S(0.5) * F[0]) * inv_rho;
  const S uy = (jy + S(0.5) * F[1]) * inv_rho;
  const S uz = D == 3 ? (jz + S(0.5) * F[2]) * inv_rho : S(0);
  if (a.u_out) {
    // Read back only after other passes have streamed through the caches.
    if constexpr (NT) {
      __builtin_nontemporal_store(ux, &a.u_out[s]);
      __builtin_nontemporal_store(uy, &a.u_out[static_cast<size_t>(g.N) + s]);
      if (D == 3) __builtin_nontemporal_store(uz, &a.u_out[2 * static_cast<size_t>(g.N) + s]);
    } else {
      a.u_out[s] = ux;
      a.u_out[static_cast<size_t>(g.N) + s] = uy;
      if (D == 3) a.u_out[2 * static_cast<size_t>(g.N) + s] = uz;
    }
  }
  if constexpr (!COLLIDE) return;

  // Ghost moments scaled by their integer basis: m_k / scale_k.
  S ghost[NR > 0 ? NR : 1];
  if constexpr (GHOST) {
    static_for<NR>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      if constexpr (k >= L::NSTRESS) {
        S m = 0;
        static_for<Q>([&](auto ic) {
          constexpr int i = decltype(ic)::value;
          constexpr int c = kIB<Q, D + 1 + k, i>;
          if constexpr (c != 0) m += S(c) * fv[i];
        });
        ghost[k] = m;
      }
    });
  }

  // Stress Pi = sum fbar Q = sum fbar c c - c_s^2 S0 I, its non-equilibrium part
  // and the Guo source T = uF + Fu, split into isotropic (bulk) and deviatoric
  // (shear) parts relaxed with gamma_b and gamma_s.
  const S cs2S0 = S(kCs2) * S0;
  const S nxx = pxx - cs2S0 - rho * ux * ux;
  const S nyy = pyy - cs2S0 - rho * uy * uy;
  const S nzz = D == 3 ? pzz - cs2S0 - rho * uz * uz : S(0);
  const S nxy = pxy - rho * ux * uy;
  const S nxz = D == 3 ? pxz - rho * ux * uz : S(0);
  const S nyz = D == 3 ? pyz - rho * uy * uz : S(0);
  const S txx = S(2) * ux * F[0], tyy = S(2) * uy * F[1], tzz = S(2) * uz * F[2];
  const S txy = ux * F[1] + F[0] * uy, txz = ux * F[2] + F[0] * uz, tyz = uy * F[2] + F[1] * uz;
  constexpr S invD = S(1.0 / D);
  const S ntr = (nxx + nyy + nzz) * invD;
  const S ttr = (txx + tyy + tzz) * invD;
  const S hs = S(0.5) * (S(1) + a.gamma_s), hb = S(0.5) * (S(1) + a.gamma_b);
  const S iso = a.gamma_b * ntr + hb * ttr;
  const S qxx = rho * ux * ux + a.gamma_s * (nxx - ntr) + hs * (txx - ttr) + iso;
  const S qyy = rho * uy * uy + a.gamma_s * (nyy - ntr) + hs * (tyy - ttr) + iso;
  const S qzz = D == 3 ? rho * uz * uz + a.gamma_s * (nzz - ntr) + hs * (tzz - ttr) + iso : S(0);
  const S qxy = rho * ux * uy + a.gamma_s * nxy + hs * txy;
  const S qxz = rho * ux * uz + a.gamma_s * nxz + hs * txz;
  const S qyz = rho * uy * uz + a.gamma_s * nyz + hs * tyz;
  const S qtr = qxx + qyy + qzz;
  const S jsx = jx + F[0], jsy = jy + F[1], jsz = jz + F[2];

  // Scale the amplitudes into integer-basis units (and add gamma_g m_g).
  static_for<NR>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr double sc = kSB<Q, D + 1 + k>;
    if constexpr (GHOST && k >= L::NSTRESS)
      nk[k] = S(sc) * (nk[k] + a.gamma_g * (S(sc) * ghost[k]));
    else
      nk[k] = S(sc) * nk[k];
  });

  static_for<Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int cx = L::cx[i], cy = L::cy[i], cz = L::cz[i];
    S cj = 0;
    if constexpr (cx != 0) cj += S(cx) * jsx;
    if constexpr (cy != 0) cj += S(cy) * jsy;
    if constexpr (cz != 0) cj += S(cz) * jsz;
    S pq = -S(kCs2) * qtr;
    if constexpr (cx != 0) pq += qxx;
    if constexpr (cy != 0) pq += qyy;
    if constexpr (cz != 0) pq += qzz;
    if constexpr (cx * cy != 0) pq += S(2 * cx * cy) * qxy;
    if constexpr (cx * cz != 0) pq += S(2 * cx * cz) * qxz;
    if constexpr (cy * cz != 0) pq += S(2 * cy * cz) * qyz;
    S nz = 0;
    static_for<NR>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr int c = kIB<Q, D + 1 + k, i>;
      if constexpr (c != 0) nz += S(c) * nk[k];
    });
    // Populations are streamed: written once here, read once by the next
    // step, so large lattices bypass the caches with them (non-temporal).
    const S fo = S(L::w[i]) * (S0 + S(3) * cj + S(4.5) * pq + nz);
    S* dst = &a.f_out[static_cast<size_t>(i) * g.N + s];
    if constexpr (NT)
      __builtin_nontemporal_store(fo, dst);
    else
      *dst = fo;
  });
}

template <typename S, bool DEV, int Q, int SMOL, bool GHOST, bool COLLIDE, bool NT,
          bool WALLS = false>
__global__ __launch_bounds__(kSiteBlock) void k_lb(LBArgs<S> a, SiteMap m) {
  int x, y, z;
  if (site_of(m, a.g, x, y, z)) lb_body<S, DEV, Q, SMOL, GHOST, COLLIDE, NT, WALLS>(a, x, y, z);
}

// ---------------------------------------------------------------------------
// z-marching tiles.  A block of kTX x kTY threads owns the columns
// [x0, x0+kTX) x [y0, y0+kTY) and the planes [z0, z1); plane-sized regions
// with an xy halo live in LDS (one plane, or a ring indexed by plane), and
// stencils that span three planes are carried from plane to plane as
// partial sums in registers.  Every global access is to a wrapped (periodic)
// coordinate; the in-plane offsets are computed once per block.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int ring(int p, int n) { return ((p % n) + n) % n; }

// ---------------------------------------------------------------------------
// Per-step preparation, z-marching: the SMOL noise N^n (Sec. V), frozen over
// the Runge-Kutta stages, and the chemical potential mu(psi^n) that the LB
// force needs.  Either part can be switched off (noise when kT = 0, mu when
// the fluid is not forced).
// ---------------------------------------------------------------------------
template <typename S>
struct PrepArgs {
  Geom g;
  Coef<S> c;
  S amp;           // sqrt(2 kT M)
  uint32_t k0, k1, step;
  int zc;
  const S* psi;    // psi^n
  S* noise;        // N^n, or nullptr
  S* mu;           // mu(psi^n), or nullptr
};

// One plane of psi for mu: region with halo 1.  The 3-D kernels carry the
// plane sums of the planes below and above in registers (SoPlanes).
template <typename S>
struct PsiPlane {
  static constexpr int W = kTX + 2, H = kTY + 2, RS = W * H;
  S v[RS];
};

// Wrapped in-plane offsets of the elements e = tid + k kTX kTY (k < NK) of a
// W-wide region whose corner is (x0 + ox, y0 + oy), computed once per block so
// that the z-marching loops do no modulo arithmetic (planes advance by one).
template <int W, int NK>
__device__ __forceinline__ void region_offsets(const Geom& g, int x0, int y0, int ox, int oy,
                                               bool near, int tid, int (&xy)[NK]) {
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int e = tid + k * kTX * kTY;
    xy[k] = wrap_r(x0 + ox + e % W, g.nx, near) + g.nx * wrap_r(y0 + oy + e / W, g.ny, near);
  }
}

__device__ __forceinline__ int next_plane(int z, int nz) { return z + 1 == nz ? 0 : z + 1; }

// psi plane at offset zoff into the region with halo 1 (offsets from
// region_offsets with corner (-1, -1)).
template <typename S>
__device__ __forceinline__ void prep_load_psi(PsiPlane<S>& r, const S* __restrict__ psi,
                                              const int (&xy)[2], int zoff, int tid) {
  static_assert(PsiPlane<S>::RS <= 2 * kTX * kTY, "two elements per thread");
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int e = tid + k * kTX * kTY;
    if (e < PsiPlane<S>::RS) r.v[e] = psi[xy[k] + zoff];
  }
}

// 2-D mu at the tile point (tx, ty).  WALLS: walls across y; a neighbour
// row beyond a wall (global row y + dy outside [0, ny)) reads the centre.
template <typename S, bool WALLS = false>
__device__ __forceinline__ S prep_mu2(const PsiPlane<S>& r, const Coef<S>& c, int tx, int ty,
                                      int y = 0, int ny = 0) {
  using R = PsiPlane<S>;
  return chem_pot<S, 2>(c, [&](int dx, int dy, int) {
    if (WALLS && (y + dy < 0 || y + dy >= ny)) return r.v[(tx + 1) + R::W * (ty + 1)];
    return r.v[(tx + 1 + dx) + R::W * (ty + 1 + dy)];
  });
}

// FV noise (Eqs. fvdiff, noiseflux, fdt_orderpara): node noise xi_a = amp z_a
// and N = Gamma . xi with Gamma = (1/c_s^2) sum_i w_i c_i.  One plane of xi
// (halo 1) lives in LDS at a time; each plane is folded into register partial
// sums of N for the planes below, at and above it.  mu(psi) comes from one
// psi plane and the plane sums of SoPlanes.
// WALLS: walls across the last axis.  3-D: a plane beyond a wall is neither
// drawn nor folded; the links across it take minus the centre's xi (a term
// +-W xi_z on the end planes) and the Laplacian the centre's psi
// (SoPlanes::mu_walled).  2-D: a link to a row beyond a wall takes minus the
// centre's xi, and the Laplacian the centre's psi.
// `plane_work(p)` runs at the start of iteration p (plane 0 in 2-D), for
// kernels that do per-plane work of their own beside the noise; MU = false
// compiles the chemical potential out (a.mu is then ignored).
struct NoPlaneWork {
  __device__ __forceinline__ void operator()(int) const {}
};

template <typename S, int Q, bool WALLS = false, bool MU = true, typename PW = NoPlaneWork>
__device__ __forceinline__ void prep_fv_body(const PrepArgs<S>& a, int bx, int by, int bz,
                                             PW plane_work = PW{}) {
  using L = Lat<Q>;
  constexpr int D = L::D;
  constexpr int W = kTX + 2, H = kTY + 2, RS = W * H;
  constexpr int NT = kTX * kTY;
  __shared__ S xi[D][RS];
  __shared__ PsiPlane<S> spsi;
  const Geom& g = a.g;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kTX + tx;
  const int x0 = bx * kTX, y0 = by * kTY;
  const bool near = g.nx >= kTX + 8 && g.ny >= kTY + 8;
  const int z0 = D == 3 ? bz * a.zc : 0, z1 = D == 3 ? min(z0 + a.zc, g.nz) : 1;
  const int x = x0 + tx, y = y0 + ty;
  const bool live = x < g.nx && y < g.ny;
  static_assert(RS <= 2 * NT, "two region elements per thread");
  int rxy[2];
  region_offsets<W>(g, x0, y0, -1, -1, near, tid, rxy);
  auto gen = [&](int zoff) {  // xi on the plane at zoff, region with halo 1
#pragma unroll 1
    for (int k = 0; k < 2; ++k) {  // not unrolled: one copy of the normal generator
      const int e = tid + k * NT;
      if (e >= RS) break;
      const uint32_t site = static_cast<uint32_t>((k ? rxy[1] : rxy[0]) + zoff);
      S zz[4];
      if constexpr (D == 2)
        Normal4<S>::gen2(site, a.step, 0, kTagSMOL, a.k0, a.k1, zz);
      else
        Normal4<S>::gen(site, a.step, 0, kTagSMOL, a.k0, a.k1, zz);
#pragma unroll
      for (int c = 0; c < D; ++c) xi[c][e] = zz[c];
    }
  };
  SoPlanes<S> so;  // psi planes p-2, p-1, p (3-D)
  S npart[3] = {0, 0, 0};  // N(p-1), N(p), N(p+1)
  auto fold = [&]() {
#pragma unroll
    for (int q = 1; q < Q; ++q) {
      int e = (tx + 1 + L::cx[q]) + W * (ty + 1 + L::cy[q]);
      bool cut = false;  // 2-D walls: the link leaves across a wall
      if constexpr (WALLS && D == 2) {
        cut = y + L::cy[q] < 0 || y + L::cy[q] >= g.ny;
        if (cut) e = (tx + 1) + W * (ty + 1);
      }
      S v = 0;
      if (L::cx[q]) v += L::cx[q] * xi[0][e];
      if (L::cy[q]) v += L::cy[q] * xi[1][e];
      if (D == 3 && L::cz[q]) v += L::cz[q] * xi[D - 1][e];
      if (cut) v = -v;
      npart[1 - L::cz[q]] += S(L::w[q]) * v;
    }
  };
  if constexpr (D == 2) {
    plane_work(0);
    if (a.noise) gen(0);
    if (MU && a.mu) prep_load_psi(spsi, a.psi, rxy, 0, tid);
    __syncthreads();
    if (a.noise) {
      fold();
      if (live) a.noise[x + g.nx * y] = S(3) * a.amp * npart[1];
    }
    if (MU && a.mu && live) a.mu[x + g.nx * y] = prep_mu2<S, WALLS>(spsi, a.c, tx, ty, y, g.ny);
  } else {
    // Iteration p: xi(p) and psi(p) staged; N(p-1) and mu(p-1) emitted.  The
    // psi plane is fetched into registers one iteration ahead.
    const int plane = g.nx * g.ny;
    int pz = wrap_any(z0 - 1, g.nz);
    S pv[2];
    auto fetch_psi = [&](int zoff) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
        if (tid + k * NT < RS) pv[k] = a.psi[rxy[k] + zoff];
    };
    if (MU && a.mu) fetch_psi(plane * pz);
    for (int p = z0 - 1; p <= z1; ++p, pz = next_plane(pz, g.nz)) {
      const bool ghost = WALLS && (p < 0 || p >= g.nz);  // a plane beyond a wall
      plane_work(p);
      if (a.noise && !ghost) gen(plane * pz);
      if (MU && a.mu) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
          if (tid + k * NT < RS) spsi.v[tid + k * NT] = pv[k];
        if (p < z1) fetch_psi(plane * next_plane(pz, g.nz));
      }
      __syncthreads();
      const bool emit = p - 1 >= z0 && p - 1 < z1;
      if (a.noise) {
        if (!ghost) fold();
        if constexpr (WALLS) {
          constexpr S kWall = S(wall_weight<Q>());
          const S xz = xi[D - 1][(tx + 1) + W * (ty + 1)];
          if (p == 0) npart[1] += kWall * xz;
          if (p == g.nz - 1) npart[1] -= kWall * xz;
        }
        if (emit && live) a.noise[x + g.nx * (y + g.ny * (p - 1))] = S(3) * a.amp * npart[0];
        npart[0] = npart[1];
        npart[1] = npart[2];
        npart[2] = 0;
      }
      if (MU && a.mu && live) {
        so.template push<W>(spsi.v + (tx + 1) + W * (ty + 1));
        if (emit)
          a.mu[x + g.nx * (y + g.ny * (p - 1))] =
              (WALLS && (p - 1 == 0 || p - 1 == g.nz - 1))
                  ? so.mu_walled(a.c, p - 1 == 0, p - 1 == g.nz - 1)
                  : so.mu(a.c);
        so.roll();
      }
      __syncthreads();
    }
  }
}

template <typename S, int Q, bool WALLS = false>
__global__ __launch_bounds__(kTX* kTY) void k_prep_fv(PrepArgs<S> a, TileMap m) {
  int bx, by, bz;
  if (tile_of(m, bx, by, bz)) prep_fv_body<S, Q, WALLS>(a, bx, by, bz);
}

// Stress-divergence force of the FV variant in 3-D (sigma and F = -G.sigma of
// k_stress and k_force_stress) in one z-marching pass, so that sigma never
// leaves the chip.  Each iteration stages a psi plane with a two-site halo in
// LDS and forms sigma, for the plane below it, on the tile with a one-site
// halo (two region elements per thread): the gradient g = 3 sum_i w_i c_i
// psi(x + c_i) as register partial sums over three planes, L_SO from the
// per-plane sums of SoPlanes.  That sigma plane goes to LDS and is folded into
// register partial sums of F: sigma at (x + c_ix, y + c_iy, q) feeds F at
// plane q - c_iz.  sigma at plane q needs psi at q-1..q+1 and F at plane z
// needs sigma at z-1..z+1, so F lags the staged psi plane by two.
template <typename S, int Q>
__global__ __launch_bounds__(kTX* kTY) void k_stress_force_fv3(Geom g, Coef<S> co,
                                                             const S* __restrict__ psi,
                                                             S* __restrict__ F, int zc,
                                                             TileMap m) {
  using L = Lat<Q>;
  static_assert(L::D == 3, "3-D lattices");
  constexpr int NS = 6, NT = kTX * kTY;
  constexpr int W1 = kTX + 2, H1 = kTY + 2, R1 = W1 * H1;  // sigma: halo 1
  constexpr int W2 = kTX + 4, H2 = kTY + 4, R2 = W2 * H2;  // psi: halo 2
  static_assert(R1 <= 2 * NT && R2 <= 2 * NT, "two region elements per thread");
  __shared__ S sp[R2];
  __shared__ S ss[NS][R1];
  int bx, by, bz;
  if (!tile_of(m, bx, by, bz)) return;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kTX + tx;
  const int x0 = bx * kTX, y0 = by * kTY;
  const bool near = g.nx >= kTX + 8 && g.ny >= kTY + 8;
  const int z0 = bz * zc, z1 = min(z0 + zc, g.nz);
  const int x = x0 + tx, y = y0 + ty;
  const bool live = x < g.nx && y < g.ny;
  int rxy[2];
  region_offsets<W2>(g, x0, y0, -2, -2, near, tid, rxy);
  // The sigma elements of this thread: e = tid + k NT < R1, centred at c2[k]
  // in the psi region.
  const int nk = tid + NT < R1 ? 2 : 1;
  int c2[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int e = tid + k * NT;
    c2[k] = (e % W1 + 1) + W2 * (e / W1 + 1);
  }
  SoPlanes<S> so[2];
  S gp[2][3][3];  // gradient partial sums of each element at planes p-1, p, p+1
  S fp[3][3];     // F partial sums at planes q-1, q, q+1 (q the folded sigma plane)
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      gp[0][j][a] = gp[1][j][a] = S(0);
      fp[j][a] = S(0);
    }
  const int plane = g.nx * g.ny;
  int pz = wrap_any(z0 - 2, g.nz);
  for (int p = z0 - 2; p <= z1 + 1; ++p, pz = next_plane(pz, g.nz)) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = tid + k * NT;
      if (e < R2) sp[e] = psi[rxy[k] + plane * pz];
    }
    __syncthreads();
    // psi(p) completes sigma(p - 1) once planes p-2, p-1 are in (p >= z0).
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k >= nk) break;
      const S* P = sp + c2[k];
      so[k].template push<W2>(P);
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const S t = S(L::w[i]) * P[L::cx[i] + W2 * L::cy[i]];
        if (L::cx[i]) gp[k][1 - L::cz[i]][0] += L::cx[i] * t;
        if (L::cy[i]) gp[k][1 - L::cz[i]][1] += L::cy[i] * t;
        if (L::cz[i]) gp[k][1 - L::cz[i]][2] += L::cz[i] * t;
      }
      if (p >= z0) {
        const int e = tid + k * NT;
        S gr[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) gr[a] = gp[k][0][a] * S(3);
        const S ps = so[k].c[1];
        const S lap = so[k].lap();
        const S g2 = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
        const S iso = S(0.5) * co.a * ps * ps + S(0.75) * co.b * ps * ps * ps * ps -
                      co.kappa * ps * lap - S(0.5) * co.kappa * g2;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = a; b < 3; ++b)
            ss[sym_idx<3>(a, b)][e] = co.kappa * gr[a] * gr[b] + (a == b ? iso : S(0));
      }
      so[k].roll();
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        gp[k][0][a] = gp[k][1][a];
        gp[k][1][a] = gp[k][2][a];
        gp[k][2][a] = S(0);
      }
    }
    __syncthreads();
    if (p >= z0) {
      // sigma(q), q = p - 1, at (x + c_ix, y + c_iy) feeds F at plane q - c_iz.
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const int e = (tx + 1 + L::cx[i]) + W1 * (ty + 1 + L::cy[i]);
        const int ci[3] = {L::cx[i], L::cy[i], L::cz[i]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          S acc = 0;
#pragma unroll
          for (int b = 0; b < 3; ++b)
            if (ci[b]) acc += ci[b] * ss[sym_idx<3>(a, b)][e];
          fp[1 - L::cz[i]][a] -= S(3) * S(L::w[i]) * acc;
        }
      }
      if (p - 2 >= z0 && p - 2 < z1 && live) {
        const int s = x + g.nx * (y + g.ny * (p - 2));
#pragma unroll
        for (int a = 0; a < 3; ++a) F[static_cast<size_t>(a) * g.N + s] = fp[0][a];
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        fp[0][a] = fp[1][a];
        fp[1][a] = fp[2][a];
        fp[2][a] = S(0);
      }
    }
  }
}

// FD noise (Sec. V.A, reading): one flux zeta_l per undirected Laplacian link,
// amplitude A_l = amp sqrt(lambda_l), N(x) = sum_l A_l [zeta_l(x - c_l) - zeta_l(x)].
// Each plane's link normals are drawn once into LDS; every thread accumulates
// its site's sums for planes p-1, p, p+1 in registers.
// plane_work and MU as for prep_fv_body.
template <typename S, int Q, bool MU = true, typename PW = NoPlaneWork>
__device__ __forceinline__ void prep_fd_body(const PrepArgs<S>& a, int bx, int by, int bz,
                                             PW plane_work = PW{}) {
  using L = Lat<Q>;
  constexpr int D = L::D;
  constexpr int NL = L::NLINKS;
  constexpr int NB = (NL + 3) / 4;
  constexpr int W = kTX + 1, H = kTY + 2, RS = W * H;  // x in [x0-1, x0+kTX), y in [y0-1, y0+kTY]
  __shared__ S zeta[NL][RS];
  __shared__ PsiPlane<S> pr;
  SoPlanes<S> so;  // psi planes p-2, p-1, p (3-D)
  const Geom& g = a.g;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kTX + tx;
  const int x0 = bx * kTX, y0 = by * kTY;
  const bool near = g.nx >= kTX + 8 && g.ny >= kTY + 8;
  const int z0 = D == 3 ? bz * a.zc : 0, z1 = D == 3 ? min(z0 + a.zc, g.nz) : 1;
  const int x = x0 + tx, y = y0 + ty;
  const bool live = x < g.nx && y < g.ny;
  S A[NL];
  static_for<NL>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    constexpr double r = ce_sqrt(L::lw[l]);
    A[l] = a.amp * S(r);
  });
  static_assert(RS <= 2 * kTX * kTY, "two region elements per thread");
  int zxy[2], pxy[2];
  region_offsets<W>(g, x0, y0, -1, -1, near, tid, zxy);
  region_offsets<PsiPlane<S>::W>(g, x0, y0, -1, -1, near, tid, pxy);
  S nm = 0, n0 = 0, np = 0;  // partial N for planes p-1, p, p+1
  const int pbeg = D == 3 ? z0 - 1 : 0, pend = D == 3 ? z1 : 0;
  const int plane = g.nx * g.ny;
  int pz = wrap_any(pbeg, g.nz);
  // the psi plane is fetched into registers one iteration ahead
  S pv[2];
  auto fetch_psi = [&](int zoff) {
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (tid + k * kTX * kTY < PsiPlane<S>::RS) pv[k] = a.psi[pxy[k] + zoff];
  };
  if (MU && a.mu) fetch_psi(plane * pz);
  for (int p = pbeg; p <= pend; ++p, pz = next_plane(pz, g.nz)) {
    plane_work(p);
    if (a.noise) {
#pragma unroll 1
      for (int k = 0; k < 2; ++k) {  // not unrolled: one copy of the normal generator
        const int e = tid + k * kTX * kTY;
        if (e >= RS) break;
        const uint32_t site = static_cast<uint32_t>((k ? zxy[1] : zxy[0]) + plane * pz);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          S zz[4];
          Normal4<S>::gen(site, a.step, b, kTagSMOL, a.k0, a.k1, zz);
#pragma unroll
          for (int l = 0; l < 4; ++l)
            if (4 * b + l < NL) zeta[4 * b + l][e] = zz[l];
        }
      }
    }
    if (MU && a.mu) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
        if (tid + k * kTX * kTY < PsiPlane<S>::RS) pr.v[tid + k * kTX * kTY] = pv[k];
      if (p < pend) fetch_psi(plane * next_plane(pz, g.nz));
    }
    __syncthreads();
    if (MU && a.mu && live) {
      if constexpr (D == 2) {
        a.mu[x + g.nx * y] = prep_mu2(pr, a.c, tx, ty);
      } else {
        so.template push<PsiPlane<S>::W>(pr.v + (tx + 1) + PsiPlane<S>::W * (ty + 1));
        if (p - 1 >= z0 && p - 1 < z1) a.mu[x + g.nx * (y + g.ny * (p - 1))] = so.mu(a.c);
        so.roll();
      }
    }
    if (live && a.noise) {
      const int own = (tx + 1) + W * (ty + 1);
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        n0 -= A[l] * zeta[l][own];
        const S in = A[l] * zeta[l][(tx + 1 - L::lx[l]) + W * (ty + 1 - L::ly[l])];
        if (L::lz[l] == 0) n0 += in;
        else if (L::lz[l] > 0) np += in;
        else nm += in;
      }
      if (D == 2) {
        a.noise[x + g.nx * y] = n0;
      } else {
        if (p - 1 >= z0 && p - 1 < z1) a.noise[x + g.nx * (y + g.ny * (p - 1))] = nm;
        nm = n0;
        n0 = np;
        np = 0;
      }
    }
    __syncthreads();
  }
}

template <typename S, int Q>
__global__ __launch_bounds__(kTX* kTY) void k_prep_fd(PrepArgs<S> a, TileMap m) {
  int bx, by, bz;
  if (tile_of(m, bx, by, bz)) prep_fd_body<S, Q>(a, bx, by, bz);
}

// The velocity pass of the streamed populations (lb_body without the
// collision: u-bar^1 for the later stages) and the SMOL noise N^n of
// prep_fv_body or prep_fd_body in one launch on the SMOL tiles (z-marching
// in 3-D).  The noise is arithmetic (the
// Box-Muller normals) and the velocity pass reads the populations with its
// vector units mostly idle, so in one kernel the two overlap.  The block of
// in-plane tile t pulls, on each of its planes, the sites t*NT ... t*NT+NT-1
// of that plane in x-fastest order (contiguous runs, read as the row blocks
// of k_lb read them; the tiles of a plane cover it); its noise keeps the
// tile's columns.  The preparation kernel then computes mu alone.
// `pull`: whether this launch forms u-bar^1 (pa.noise null: no noise).
template <typename S, bool DEV, int Q, int SMOL, bool NT, bool WALLS>
__device__ __forceinline__ void uend_noise_body(const LBArgs<S>& la, const PrepArgs<S>& pa,
                                                bool pull, int bx, int by, int bz) {
  constexpr int D = Lat<Q>::D;
  const Geom& g = la.g;
  const int ntx = (g.nx + kTX - 1) / kTX;
  const int z0 = D == 3 ? bz * pa.zc : 0, z1 = D == 3 ? min(z0 + pa.zc, g.nz) : 1;
  const int e = (bx + ntx * by) * (kTX * kTY) + threadIdx.y * kTX + threadIdx.x;
  const bool pulls = pull && e < g.nx * g.ny;
  const int x = pulls ? e % g.nx : 0, y = pulls ? e / g.nx : 0;
  auto work = [&](int p) {
    if (pulls && p >= z0 && p < z1) lb_body<S, DEV, Q, SMOL, false, false, NT, WALLS>(la, x, y, p);
  };
  if constexpr (SMOL == kFV)
    prep_fv_body<S, Q, WALLS, false>(pa, bx, by, bz, work);
  else
    prep_fd_body<S, Q, false>(pa, bx, by, bz, work);
}

template <typename S, bool DEV, int Q, int SMOL, bool NT, bool WALLS = false>
__global__ __launch_bounds__(kTX* kTY) void k_uend_noise(LBArgs<S> la, PrepArgs<S> pa, TileMap m) {
  int bx, by, bz;
  if (tile_of(m, bx, by, bz))
    uend_noise_body<S, DEV, Q, SMOL, NT, WALLS>(la, pa, true, bx, by, bz);
}

// ---------------------------------------------------------------------------
// FD noise built in Fourier space (Sec. V.A, Eq. etafdt):
//   N = F^-1[ sqrt(-2 kT M L_SO(q)) F[w] ],  w(x) = normal slot 0 (SMOL stream).
// The transforms are hipFFT's real-to-complex pair (half spectrum of
// nz x ny x (nx/2 + 1) values, x fastest); these kernels draw w, build the
// amplitude table once (the 1/N of the unnormalised inverse folded in) and
// apply it to the spectrum.
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(256) void k_white(int n, uint32_t step, uint32_t k0, uint32_t k1,
                                               S* __restrict__ w) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  S z[4];
  Normal4<S>::gen2(static_cast<uint32_t>(s), step, 0, kTagSMOL, k0, k1, z);
  w[s] = z[0];
}

// Symbol of the Shinozaki-Oono Laplacian: Eq. (solapft) in 3-D,
// cos q_x + cos q_y + cos q_x cos q_y - 3 in 2-D.
template <typename S, int D>
__global__ __launch_bounds__(256) void k_fourier_amp(Geom g, double two_kT_M,
                                                     S* __restrict__ amp) {
  const int hx = g.nx / 2 + 1;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= hx * g.ny * g.nz) return;
  const int kx = i % hx, ky = (i / hx) % g.ny, kz = i / (hx * g.ny);
  const double cx = cospi(2.0 * kx / g.nx), cy = cospi(2.0 * ky / g.ny);
  double L;
  if constexpr (D == 3) {
    const double cz = cospi(2.0 * kz / g.nz);
    L = (12.0 * (cx + cy + cz) + 12.0 * (cx * cy + cx * cz + cy * cz) + 8.0 * cx * cy * cz -
         80.0) / 22.0;
  } else {
    L = cx + cy + cx * cy - 3.0;
  }
  const double v = -two_kT_M * L;
  amp[i] = S((v > 0.0 ? sqrt(v) : 0.0) / static_cast<double>(g.N));
}

// acc[i] += |spec[i]|^2 * scale in FP64 (whole-zone structure factor).
template <typename S>
__global__ __launch_bounds__(256) void k_power_acc(int nh, const S* __restrict__ spec,
                                                   double scale, double* __restrict__ acc) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nh) return;
  const double re = spec[2 * static_cast<size_t>(i)], im = spec[2 * static_cast<size_t>(i) + 1];
  acc[i] += (re * re + im * im) * scale;
}

// spec[i] *= amp[i] on the interleaved (re, im) half spectrum.
template <typename S>
__global__ __launch_bounds__(256) void k_fourier_scale(int nh, const S* __restrict__ amp,
                                                       S* __restrict__ spec) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nh) return;
  const S a = amp[i];
  spec[2 * static_cast<size_t>(i)] *= a;
  spec[2 * static_cast<size_t>(i) + 1] *= a;
}

// ---------------------------------------------------------------------------
// One SMOL Runge-Kutta stage with frozen u^n and N^n (Sec. V):
//   G(phi) = -Div(u phi) + M L_out mu(phi) + N.
// Combination: mode kComb: out = psi_n + cnext G (and acc update when
// acc != nullptr: acc = (first ? 0 : acc) + cacc G, or on the last stage
// out = psi_n + acc + cacc G); mode kHeun2: out = (psi_n + phi + G) / 2.
// ---------------------------------------------------------------------------
enum : int { kComb = 0, kHeun2 = 1 };
enum : int { kAtN = 0, kAtN1 = 1, kAtMid = 2 };

template <typename S>
struct StageArgs {
  Geom g;
  Coef<S> c;
  const S* phi;    // stage input
  const S* u;      // u^n (d*N) or nullptr when the flow is uniform
  const S* u_end;  // velocity of the streamed populations at t_{n+1} (d*N)
  int utime;       // stage time level: kAtN (u), kAtN1 (u_end), kAtMid (their mean)
  S u0, u1, u2;    // uniform imposed flow (SMOL_ONLY)
  const S* noise;  // N^n
  const S* psi_n;
  S* out;
  S* acc;
  S cnext, cacc;
  int mode, first, last;
  int zc;
};

template <typename S>
__device__ __forceinline__ void combine(const StageArgs<S>& a, int s, S G) {
  if (a.mode == kHeun2) {
    a.out[s] = S(0.5) * (a.psi_n[s] + a.phi[s] + G);
    return;
  }
  if (a.acc == nullptr) {
    a.out[s] = a.psi_n[s] + a.cnext * G;
    return;
  }
  const S prev = a.first ? S(0) : a.acc[s];
  if (a.last) {
    a.out[s] = a.psi_n[s] + prev + a.cacc * G;
  } else {
    a.out[s] = a.psi_n[s] + a.cnext * G;
    a.acc[s] = prev + a.cacc * G;
  }
}

// Advecting velocity of the stage: each Runge-Kutta stage sees the velocity
// of its own time level (only the noise is frozen over the step).
template <typename S>
__device__ __forceinline__ S uval(const StageArgs<S>& a, int comp, int site) {
  if (!a.u) return comp == 0 ? a.u0 : (comp == 1 ? a.u1 : a.u2);
  const size_t k = static_cast<size_t>(comp) * a.g.N + site;
  if (a.utime == kAtN) return a.u[k];
  if (a.utime == kAtN1) return a.u_end[k];
  return S(0.5) * (a.u[k] + a.u_end[k]);
}

// Values of one site that the stage's combination reads, fetched early so the
// loads overlap the stencil work of the same plane.
template <typename S>
struct SiteIn {
  S noise, psi_n, phi, acc;
};

template <typename S>
__device__ __forceinline__ SiteIn<S> fetch_site(const StageArgs<S>& a, int s) {
  SiteIn<S> v;
  v.noise = a.noise[s];
  v.psi_n = a.psi_n[s];
  v.phi = a.mode == kHeun2 ? a.phi[s] : S(0);
  v.acc = (a.acc && !a.first) ? a.acc[s] : S(0);
  return v;
}

template <typename S>
__device__ __forceinline__ void combine_in(const StageArgs<S>& a, int s, S G, const SiteIn<S>& v) {
  if (a.mode == kHeun2) {
    a.out[s] = S(0.5) * (v.psi_n + v.phi + G);
  } else if (a.acc == nullptr) {
    a.out[s] = v.psi_n + a.cnext * G;
  } else if (a.last) {
    a.out[s] = v.psi_n + v.acc + a.cacc * G;
  } else {
    a.out[s] = v.psi_n + a.cnext * G;
    a.acc[s] = v.acc + a.cacc * G;
  }
}

// Stage forms fixed at compile time, so that the z-marching loop carries no
// uniform branches on the velocity's time level or the combination: the two
// stages of Heun's method under full coupling.  kStageAny reads them from the
// arguments.
enum : int { kStageAny = 0, kStageHeun1 = 1, kStageHeun2 = 2 };

template <int SF, typename S>
__device__ __forceinline__ S uval_sf(const StageArgs<S>& a, int comp, int site) {
  const size_t k = static_cast<size_t>(comp) * a.g.N + site;
  if constexpr (SF == kStageHeun1)
    return a.u[k];
  else if constexpr (SF == kStageHeun2)
    return a.u_end[k];
  else
    return uval(a, comp, site);
}

template <int SF, typename S>
__device__ __forceinline__ SiteIn<S> fetch_site_sf(const StageArgs<S>& a, int s) {
  if constexpr (SF == kStageAny) {
    return fetch_site(a, s);
  } else {
    SiteIn<S> v;
    v.noise = a.noise[s];
    v.psi_n = a.psi_n[s];
    v.phi = SF == kStageHeun2 ? a.phi[s] : S(0);
    v.acc = S(0);
    return v;
  }
}

template <int SF, typename S>
__device__ __forceinline__ void combine_sf(const StageArgs<S>& a, int s, S G, const SiteIn<S>& v) {
  if constexpr (SF == kStageHeun1)
    a.out[s] = v.psi_n + a.cnext * G;
  else if constexpr (SF == kStageHeun2)
    a.out[s] = S(0.5) * (v.psi_n + v.phi + G);
  else
    combine_in(a, s, G, v);
}

// FV stage (Sec. V.B, Eq. fvft): G = Gamma . J + N with the node flux
// J = -u phi + M Gamma mu(phi).  2-D: one plane, phi (halo 3), mu (halo 2)
// and J (halo 1) in LDS, one phase each.
// WALLS: walls across y; mu and Gamma mu read the centre's value across a
// wall, Gamma . J minus the centre's J.
template <typename S, int Q, bool WALLS = false>
__device__ __forceinline__ void stage_fv2_body(const StageArgs<S>& a, int bx, int by) {
  using L = Lat<Q>;
  constexpr int D = L::D;
  constexpr int WP = kTX + 6, HP = kTY + 6;
  constexpr int WM = kTX + 4, HM = kTY + 4;
  constexpr int WJ = kTX + 2, HJ = kTY + 2;
  constexpr int NT = kTX * kTY;
  __shared__ S sphi[WP * HP];
  __shared__ S smu[WM * HM];
  __shared__ S sJ[D][WJ * HJ];
  const Geom& g = a.g;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kTX + tx;
  const int x0 = bx * kTX, y0 = by * kTY;
  const bool near = g.nx >= kTX + 8 && g.ny >= kTY + 8;
  const int x = x0 + tx, y = y0 + ty;
  const bool live = x < g.nx && y < g.ny;
  SiteIn<S> sv{};
  if (live) sv = fetch_site(a, x + g.nx * y);
  for (int e = tid; e < WP * HP; e += NT) {
    const int i = e % WP, j = e / WP;
    sphi[e] = a.phi[wrap_r(x0 - 3 + i, g.nx, near) + g.nx * wrap_r(y0 - 3 + j, g.ny, near)];
  }
  __syncthreads();
  for (int e = tid; e < WM * HM; e += NT) {
    const int i = e % WM, j = e / WM;
    const int yr = y0 - 2 + j;  // global row of this mu point
    smu[e] = chem_pot<S, D>(a.c, [&](int dx, int dy, int) {
      if (WALLS && (yr + dy < 0 || yr + dy >= g.ny)) return sphi[(i + 1) + WP * (j + 1)];
      return sphi[(i + 1 + dx) + WP * (j + 1 + dy)];
    });
  }
  __syncthreads();
  for (int e = tid; e < WJ * HJ; e += NT) {
    const int i = e % WJ, j = e / WJ;
    const int site = wrap_r(x0 - 1 + i, g.nx, near) + g.nx * wrap_r(y0 - 1 + j, g.ny, near);
    const int yr = y0 - 1 + j;  // global row of this J point
    S gm[2] = {0, 0};
#pragma unroll
    for (int q = 1; q < Q; ++q) {
      const bool cut = WALLS && (yr + L::cy[q] < 0 || yr + L::cy[q] >= g.ny);
      const S t = S(L::w[q]) * (cut ? smu[(i + 1) + WM * (j + 1)]
                                    : smu[(i + 1 + L::cx[q]) + WM * (j + 1 + L::cy[q])]);
      if (L::cx[q]) gm[0] += L::cx[q] * t;
      if (L::cy[q]) gm[1] += L::cy[q] * t;
    }
    const S ph = sphi[(i + 2) + WP * (j + 2)];
#pragma unroll
    for (int c = 0; c < D; ++c) sJ[c][e] = -uval(a, c, site) * ph + a.c.M * (S(3) * gm[c]);
  }
  __syncthreads();
  S G = 0;
#pragma unroll
  for (int q = 1; q < Q; ++q) {
    const bool cut = WALLS && (y + L::cy[q] < 0 || y + L::cy[q] >= g.ny);
    const int e = cut ? (tx + 1) + WJ * (ty + 1) : (tx + 1 + L::cx[q]) + WJ * (ty + 1 + L::cy[q]);
    S v = 0;
    if (L::cx[q]) v += L::cx[q] * sJ[0][e];
    if (L::cy[q]) v += L::cy[q] * sJ[1][e];
    G += S(L::w[q]) * (cut ? -v : v);
  }
  if (live) combine_in(a, x + g.nx * y, S(3) * G + sv.noise, sv);
}

// 3-D: z-marching with one LDS plane of phi (halo 3), a three-plane ring of mu
// (halo 2) and one plane of J (halo 1).  mu comes from per-plane sums of phi
// carried in registers (SoPlanes), so each phi value in LDS is read 9 times
// instead of 27.
// Gamma . J of the G points is folded plane by plane into register partial
// sums for the planes below, at and above (a tap with z-velocity cz reaches
// the plane z - cz).  A thread owns fixed points of the mu region (index
// e = tid + k NT in a (kTX+4) x (kTY+4) layout; J lives on its inner ring) and
// one G point; iteration p loads phi(p) and emits mu(p-1), J(p-2), G(p-3).
// WALLS: walls across z.  The Laplacian and Gamma mu take the centre's value
// beyond a wall; a J plane beyond a wall is not folded, and the links across
// it take minus the centre's J (a term +-W J_z on the end planes).
template <typename S, int Q, bool WALLS = false, int SF = kStageAny>
__device__ __forceinline__ void stage_fv3_body(const StageArgs<S>& a, int bx, int by, int bz) {
  using L = Lat<Q>;
  constexpr int D = 3;
  constexpr int WP = kTX + 6, HP = kTY + 6;  // phi region
  constexpr int WM = kTX + 4, HM = kTY + 4;  // mu region; J on its inner ring
  constexpr int NT = kTX * kTY;
  constexpr int NPF = (WP * HP + NT - 1) / NT;
  constexpr int NE = (WM * HM + NT - 1) / NT;
  // FP64: the elements every thread owns are known at compile time (fewer
  // masked branches; measured 5% faster).  FP32 keeps the run-time test,
  // which measured 6% faster there.
  constexpr bool kFixed = sizeof(S) == 8;
  __shared__ S sphi[WP * HP];
  __shared__ S smu[3][WM * HM];
  __shared__ S sJ[D][WM * HM];
  const Geom& g = a.g;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kTX + tx;
  const int x0 = bx * kTX, y0 = by * kTY;
  const bool near = g.nx >= kTX + 8 && g.ny >= kTY + 8;
  const int z0 = bz * a.zc;
  const int z1 = min(z0 + a.zc, g.nz);
  const int x = x0 + tx, y = y0 + ty;
  const bool live = x < g.nx && y < g.ny;
  const int plane = g.nx * g.ny;

  int pxy[NE];
  bool pon[NE], jon[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = tid + k * NT;
    const int i = e % WM, j = e / WM;
    pon[k] = (kFixed && (k + 1) * NT <= WM * HM) || e < WM * HM;
    jon[k] = pon[k] && i >= 1 && i < WM - 1 && j >= 1 && j < HM - 1;
    pxy[k] = wrap_r(x0 - 2 + i, g.nx, near) + g.nx * wrap_r(y0 - 2 + j, g.ny, near);
  }

  // In-plane offsets of the phi elements this thread loads; the planes are
  // tracked incrementally, so the loop does no modulo arithmetic.
  int fxy[NPF];
#pragma unroll
  for (int k = 0; k < NPF; ++k) {
    const int e = tid + k * NT;
    fxy[k] = wrap_r(x0 - 3 + e % WP, g.nx, near) + g.nx * wrap_r(y0 - 3 + e / WP, g.ny, near);
  }
  S pf[NPF];
  auto fetch_phi = [&](int zoff) {
#pragma unroll
    for (int k = 0; k < NPF; ++k)
      if ((kFixed && (k + 1) * NT <= WP * HP) || tid + k * NT < WP * HP)
        pf[k] = a.phi[fxy[k] + zoff];
  };

  SoPlanes<S> so[NE];                  // phi planes p-2, p-1, p
  S uv[NE][D];
  S gpart[3] = {0, 0, 0};              // G planes p-3, p-2, p-1
#pragma unroll
  for (int k = 0; k < NE; ++k)
#pragma unroll
    for (int c = 0; c < D; ++c) uv[k][c] = 0;

  int zf = wrap_any(z0 - 3, g.nz);  // plane of the phi fetch
  int zu = wrap_any(z0 - 5, g.nz);  // plane p - 2 of the velocity at iteration p
  fetch_phi(plane * zf);
  for (int p = z0 - 3; p <= z1 + 2; ++p) {
    const bool do_mu = p >= z0 - 1, do_J = p >= z0 + 1, do_G = p >= z0 + 3 && live;
#pragma unroll
    for (int k = 0; k < NPF; ++k)
      if ((kFixed && (k + 1) * NT <= WP * HP) || tid + k * NT < WP * HP)
        sphi[tid + k * NT] = pf[k];
    zf = next_plane(zf, g.nz);
    if (p < z1 + 2) fetch_phi(plane * zf);
    const int s = x + g.nx * (y + g.ny * (p - 3));
    SiteIn<S> sv{};
    if (do_G) sv = fetch_site_sf<SF>(a, s);
    if (do_J) {
      const int zo = plane * zu;
#pragma unroll
      for (int k = 0; k < NE; ++k)
        if (jon[k]) {
#pragma unroll
          for (int c = 0; c < D; ++c) uv[k][c] = uval_sf<SF>(a, c, pxy[k] + zo);
        }
    }
    zu = next_plane(zu, g.nz);
    __syncthreads();
    // Plane sums of phi(p); mu(p-1) from planes p-2, p-1, p.
    const int mslot = ring(p - 1, 3);
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      if (!pon[k]) continue;
      const int e = tid + k * NT;
      so[k].template push<WP>(sphi + (e % WM + 1) + WP * (e / WM + 1));
      if (do_mu)
        smu[mslot][e] = (WALLS && (p - 1 == 0 || p - 1 == g.nz - 1))
                            ? so[k].mu_walled(a.c, p - 1 == 0, p - 1 == g.nz - 1)
                            : so[k].mu(a.c);
    }
    __syncthreads();
    // J(p-2) from mu(p-3), mu(p-2), mu(p-1).
    if (do_J) {
      const bool jlo = WALLS && p - 2 == 0, jhi = WALLS && p - 2 == g.nz - 1;
#pragma unroll
      for (int k = 0; k < NE; ++k) {
        if (!jon[k]) continue;
        const int e = tid + k * NT;
        S gm[3] = {0, 0, 0};
        if (WALLS && (jlo || jhi)) {
          // an end plane: the links across the wall read the centre's mu
#pragma unroll
          for (int q = 1; q < Q; ++q) {
            const bool cut = (jlo && L::cz[q] < 0) || (jhi && L::cz[q] > 0);
            const S t = S(L::w[q]) * (cut ? smu[ring(p - 2, 3)][e]
                                          : smu[ring(p - 2 + L::cz[q], 3)]
                                               [e + L::cx[q] + WM * L::cy[q]]);
            if (L::cx[q]) gm[0] += L::cx[q] * t;
            if (L::cy[q]) gm[1] += L::cy[q] * t;
            if (L::cz[q]) gm[2] += L::cz[q] * t;
          }
        } else {
#pragma unroll
          for (int q = 1; q < Q; ++q) {
            const S t = S(L::w[q]) * smu[ring(p - 2 + L::cz[q], 3)][e + L::cx[q] + WM * L::cy[q]];
            if (L::cx[q]) gm[0] += L::cx[q] * t;
            if (L::cy[q]) gm[1] += L::cy[q] * t;
            if (L::cz[q]) gm[2] += L::cz[q] * t;
          }
        }
        const S ph = so[k].c[0];  // phi(p-2)
#pragma unroll
        for (int c = 0; c < D; ++c) sJ[c][e] = -uv[k][c] * ph + a.c.M * (S(3) * gm[c]);
      }
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) so[k].roll();
    __syncthreads();
    // Gamma . J(p-2) into the G partials; G(p-3) complete.
    if (do_J) {
      if (!(WALLS && (p - 2 < 0 || p - 2 >= g.nz))) {
#pragma unroll
        for (int q = 1; q < Q; ++q) {
          const int e = (tx + 2 + L::cx[q]) + WM * (ty + 2 + L::cy[q]);
          S v = 0;
          if (L::cx[q]) v += L::cx[q] * sJ[0][e];
          if (L::cy[q]) v += L::cy[q] * sJ[1][e];
          if (L::cz[q]) v += L::cz[q] * sJ[2][e];
          gpart[1 - L::cz[q]] += S(L::w[q]) * v;
        }
      }
      if constexpr (WALLS) {
        constexpr S kWall = S(wall_weight<Q>());
        const S jz = sJ[2][(tx + 2) + WM * (ty + 2)];
        if (p - 2 == 0) gpart[1] += kWall * jz;
        if (p - 2 == g.nz - 1) gpart[1] -= kWall * jz;
      }
      if (do_G) combine_sf<SF>(a, s, S(3) * gpart[0] + sv.noise, sv);
      gpart[0] = gpart[1];
      gpart[1] = gpart[2];
      gpart[2] = 0;
    }
  }
}

template <typename S, int Q, bool WALLS = false, int SF = kStageAny>
__device__ __forceinline__ void stage_fv_body(const StageArgs<S>& a, int bx, int by, int bz) {
  if constexpr (Lat<Q>::D == 3)
    stage_fv3_body<S, Q, WALLS, SF>(a, bx, by, bz);
  else
    stage_fv2_body<S, Q, WALLS>(a, bx, by);
}

template <typename S, int Q, bool WALLS = false, int SF = kStageAny>
__global__ __launch_bounds__(kTX* kTY) void k_stage_fv(StageArgs<S> a, TileMap m) {
  int bx, by, bz;
  if (tile_of(m, bx, by, bz)) stage_fv_body<S, Q, WALLS, SF>(a, bx, by, bz);
}

// FD stage (Sec. V.A): G = -D.(u phi) + M L_SO mu(phi) + N with the central
// divergence D.  Rings: phi (halo 2, 5 planes), mu (halo 1, 3 planes).
template <typename S, int Q>
__device__ __forceinline__ void stage_fd_body(const StageArgs<S>& a, int bx, int by, int bz) {
  using L = Lat<Q>;
  constexpr int D = L::D;
  constexpr int WP = kTX + 4, HP = kTY + 4;
  constexpr int WM = kTX + 2, HM = kTY + 2;
  constexpr int NP = D == 3 ? 5 : 1, NM = D == 3 ? 3 : 1;
  constexpr int NT = kTX * kTY;
  __shared__ S sphi[NP][WP * HP];
  __shared__ S smu[NM][WM * HM];
  const Geom& g = a.g;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kTX + tx;
  const int x0 = bx * kTX, y0 = by * kTY;
  const bool near = g.nx >= kTX + 8 && g.ny >= kTY + 8;
  const int z0 = D == 3 ? bz * a.zc : 0;
  const int z1 = D == 3 ? min(z0 + a.zc, g.nz) : 1;

  static_assert(WP * HP <= 2 * NT, "two region elements per thread");
  int fxy[2];
  region_offsets<WP>(g, x0, y0, -2, -2, near, tid, fxy);
  const int plane = g.nx * g.ny;
  auto load_phi = [&](int p, int pz) {
    const int slot = ring(p, NP);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = tid + k * NT;
      if (e < WP * HP) sphi[slot][e] = a.phi[fxy[k] + plane * pz];
    }
  };
  auto comp_mu = [&](int p) {
    const int slot = ring(p, NM);
    for (int e = tid; e < WM * HM; e += NT) {
      const int i = e % WM, j = e / WM;
      smu[slot][e] = chem_pot<S, D>(a.c, [&](int dx, int dy, int dz) {
        return sphi[ring(p + dz, NP)][(i + 1 + dx) + WP * (j + 1 + dy)];
      });
    }
  };
  auto comp_G = [&](int t) {
    const int x = x0 + tx, y = y0 + ty;
    if (x >= g.nx || y >= g.ny) return;
    const Nbr nb(g, x, y, t);
    auto ph = [&](int dx, int dy, int dz) {
      return sphi[ring(t + dz, NP)][(tx + 2 + dx) + WP * (ty + 2 + dy)];
    };
    S adv = S(0.5) * (uval(a, 0, nb.at(1, 0, 0)) * ph(1, 0, 0) -
                      uval(a, 0, nb.at(-1, 0, 0)) * ph(-1, 0, 0)) +
            S(0.5) * (uval(a, 1, nb.at(0, 1, 0)) * ph(0, 1, 0) -
                      uval(a, 1, nb.at(0, -1, 0)) * ph(0, -1, 0));
    if (D == 3)
      adv += S(0.5) * (uval(a, 2, nb.at(0, 0, 1)) * ph(0, 0, 1) -
                       uval(a, 2, nb.at(0, 0, -1)) * ph(0, 0, -1));
    const S lap = lap_so<S, D>([&](int dx, int dy, int dz) {
      return smu[ring(t + dz, NM)][(tx + 1 + dx) + WM * (ty + 1 + dy)];
    });
    const int s = nb.at(0, 0, 0);
    combine(a, s, -adv + a.c.M * lap + a.noise[s]);
  };

  if constexpr (D == 2) {
    load_phi(0, 0);
    __syncthreads();
    comp_mu(0);
    __syncthreads();
    comp_G(0);
  } else {
    int pz = wrap_any(z0 - 2, g.nz);
    for (int t = z0 - 4; t < z1; ++t, pz = next_plane(pz, g.nz)) {
      load_phi(t + 2, pz);
      __syncthreads();
      if (t + 1 >= z0 - 1) comp_mu(t + 1);
      __syncthreads();
      if (t >= z0) comp_G(t);
    }
  }
}

template <typename S, int Q>
__global__ __launch_bounds__(kTX* kTY) void k_stage_fd(StageArgs<S> a, TileMap m) {
  int bx, by, bz;
  if (tile_of(m, bx, by, bz)) stage_fd_body<S, Q>(a, bx, by, bz);
}

// mu(phi) between walls across the last axis, one thread per site (the k_mu
// grid): a neighbour beyond a wall reads the centre's value.  The velocity
// observable takes its force from it; the step computes mu in the tiled
// kernels.
template <typename S, int Q>
__global__ __launch_bounds__(kBX* kBY) void k_mu_w(Geom g, Coef<S> c, const S* __restrict__ phi,
                                                   S* __restrict__ mu) {
  constexpr int D = Lat<Q>::D;
  const int x = blockIdx.x * kBX + threadIdx.x, y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const Nbr nb(g, x, y, z);
  const int s = nb.at(0, 0, 0);
  mu[s] = chem_pot<S, D>(c, [&](int dx, int dy, int dz) {
    return beyond_wall<D>(g, y, z, dy, dz) ? phi[s] : phi[nb.at(dx, dy, dz)];
  });
}


// ---------------------------------------------------------------------------
// Initial state and observables (one thread per site, 1-D grid).
// ---------------------------------------------------------------------------
// Diagnostics: normals of Philox blocks 0 .. nblk-1 at sites site0 + i,
// written as FP64 [site][slot] (slots beyond nslots dropped).
template <typename S>
__global__ __launch_bounds__(256) void k_diag_normals(uint32_t site0, int n, int nslots, uint32_t step,
                                                       uint32_t tag, uint32_t k0, uint32_t k1,
                                                       double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int b = 0; 4 * b < nslots; ++b) {
    S z[4];
    Normal4<S>::gen(site0 + static_cast<uint32_t>(i), step, static_cast<uint32_t>(b), tag, k0, k1, z);
    for (int l = 0; l < 4 && 4 * b + l < nslots; ++l)
      out[static_cast<size_t>(i) * nslots + 4 * b + l] = static_cast<double>(z[l]);
  }
}

// psi^0 = std z + profile; profile = psi_eq [tanh((h - L/4)/l) - tanh((h - 3L/4)/l) - 1]
// along the last axis when tanh_on.
template <typename S, int Q>
__global__ __launch_bounds__(256) void k_init_psi(Geom g, double std_, int tanh_on, double psi_eq,
                                                  double l, uint32_t k0, uint32_t k1,
                                                  S* __restrict__ psi) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  double z2[2];
  Normal4<double>::gen2(static_cast<uint32_t>(s), 0u, 0u, kTagInit, k0, k1, z2);
  double v = std_ * z2[0];
  if (tanh_on) {
    const int h = Lat<Q>::D == 3 ? s / (g.nx * g.ny) : (s / g.nx) % g.ny;
    const double Lh = Lat<Q>::D == 3 ? g.nz : g.ny;
    v += psi_eq * (tanh((h - 0.25 * Lh) / l) - tanh((h - 0.75 * Lh) / l) - 1.0);
  }
  psi[s] = static_cast<S>(v);
}

// Walls across the last axis for the kernels that convert between the
// stored post-collision populations and the streamed ones (on = 0: periodic).
struct WallSpec {
  int on;
  double rho0;
  double u[2][3];  // velocities of the lower and upper wall
};

// fbar_i at site s = (x, y, z): f*_i(x - c_i) as the next step's streaming
// pulls it, or, where x - c_i lies beyond a wall, the site's own reversed
// f*_opp(i) plus the moving-wall term 6 w_i rho0 c_i.U (the same rule as the
// bounce-back pull of the LB kernel).  FP64, stored units (deviations when
// the populations are stored as deviations).
template <typename S, int Q>
__device__ __forceinline__ double streamed_pop(const Geom& g, const WallSpec& w,
                                               const S* __restrict__ f, const Nbr& nb, int s,
                                               int y, int z, int i) {
  using L = Lat<Q>;
  if (w.on && beyond_wall<L::D>(g, y, z, -L::cy[i], -L::cz[i])) {
    const double* U = c_last<Q>(i) > 0 ? w.u[0] : w.u[1];
    double cU = 0;
    if (L::cx[i]) cU += L::cx[i] * U[0];
    if (L::cy[i]) cU += L::cy[i] * U[1];
    if (L::cz[i]) cU += L::cz[i] * U[2];
    return static_cast<double>(f[static_cast<size_t>(kOpp<Q>.i[i]) * g.N + s]) +
           6.0 * L::w[i] * w.rho0 * cU;
  }
  return static_cast<double>(
      f[static_cast<size_t>(i) * g.N + nb.at(-L::cx[i], -L::cy[i], -L::cz[i])]);
}

// Stored f*(x) = fbar(x + c_i) for a user fbar given in FP64; the inverse of
// streamed_pop: where x + c_i lies beyond a wall, f*_i(x) = fbar_opp(i)(x) +
// 6 w_i rho0 c_i.U of the wall that c_i points into.
template <typename S, bool DEV, int Q>
__global__ __launch_bounds__(256) void k_scatter_user(Geom g, WallSpec w,
                                                      const double* __restrict__ fin,
                                                      S* __restrict__ f) {
  using L = Lat<Q>;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const int x = s % g.nx, y = (s / g.nx) % g.ny, z = s / (g.nx * g.ny);
  const Nbr nb(g, x, y, z);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    double v;
    if (w.on && beyond_wall<L::D>(g, y, z, L::cy[i], L::cz[i])) {
      const double* U = c_last<Q>(i) < 0 ? w.u[0] : w.u[1];
      double cU = 0;
      if (L::cx[i]) cU += L::cx[i] * U[0];
      if (L::cy[i]) cU += L::cy[i] * U[1];
      if (L::cz[i]) cU += L::cz[i] * U[2];
      v = fin[static_cast<size_t>(kOpp<Q>.i[i]) * g.N + s] + 6.0 * L::w[i] * w.rho0 * cU;
    } else {
      v = fin[static_cast<size_t>(i) * g.N + nb.at(L::cx[i], L::cy[i], L::cz[i])];
    }
    f[static_cast<size_t>(i) * g.N + s] = static_cast<S>(DEV ? v - L::w[i] * w.rho0 : v);
  }
}

// Uniform start: the streamed populations are the equilibrium of (rho0, u)
// at every site.  Stored f*_i(x) = f^eq_i, except where x + c_i lies beyond a
// wall: there the next pull bounces f*_i back into fbar_opp(i)(x), so f*_i =
// f^eq_opp(i) + 6 w_i rho0 c_i.U (as k_scatter_user).
template <typename S, bool DEV, int Q>
__global__ __launch_bounds__(256) void k_init_uniform(Geom g, WallSpec w, double ux, double uy,
                                                      double uz, S* __restrict__ f) {
  using L = Lat<Q>;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const int y = (s / g.nx) % g.ny, z = s / (g.nx * g.ny);
  const double rho0 = w.rho0;
  const double usq = ux * ux + uy * uy + uz * uz;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const bool out = w.on && beyond_wall<L::D>(g, y, z, L::cy[i], L::cz[i]);
    const int j = out ? kOpp<Q>.i[i] : i;
    const double cu = L::cx[j] * ux + L::cy[j] * uy + L::cz[j] * uz;
    double fe = L::w[j] * rho0 * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
    if (out) {
      const double* U = c_last<Q>(i) < 0 ? w.u[0] : w.u[1];
      double cU = 0;
      if (L::cx[i]) cU += L::cx[i] * U[0];
      if (L::cy[i]) cU += L::cy[i] * U[1];
      if (L::cz[i]) cU += L::cz[i] * U[2];
      fe += 6.0 * L::w[i] * rho0 * cU;
    }
    f[static_cast<size_t>(i) * g.N + s] = static_cast<S>(DEV ? fe - L::w[i] * rho0 : fe);
  }
}

// fbar(x) (streamed_pop), in FP64 (+ w_i rho0 for deviations); rho optional.
template <typename S, bool DEV, int Q>
__global__ __launch_bounds__(256) void k_gather(Geom g, WallSpec w, const S* __restrict__ f,
                                                double* __restrict__ pop,
                                                double* __restrict__ rho) {
  using L = Lat<Q>;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const int x = s % g.nx, y = (s / g.nx) % g.ny, z = s / (g.nx * g.ny);
  const Nbr nb(g, x, y, z);
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    double v = streamed_pop<S, Q>(g, w, f, nb, s, y, z, i);
    if (DEV) v += L::w[i] * w.rho0;
    if (pop) pop[static_cast<size_t>(i) * g.N + s] = v;
    r += v;
  }
  if (rho) rho[s] = r;
}

// Element counts up to d*N exceed 2^31 on the largest lattices: 64-bit
// indices.
template <typename S>
__global__ __launch_bounds__(256) void k_to_f64(int64_t n, const S* __restrict__ in,
                                                double* __restrict__ out) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s < n) out[s] = static_cast<double>(in[s]);
}

template <typename S>
__global__ __launch_bounds__(256) void k_from_f64(int64_t n, const double* __restrict__ in,
                                                  S* __restrict__ out) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s < n) out[s] = static_cast<S>(in[s]);
}

// Zero n 32-bit words: a kernel rather than a memset, so that a caller may
// capture the clear into a graph.
__global__ __launch_bounds__(256) void k_zero_words(int64_t n, uint32_t* __restrict__ p) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Totals in FP64: per-block partials of (rho, j, psi, |rho|, |j|, |psi|),
// then one block sums the partials in a fixed order (deterministic).
constexpr int kTotBlock = 256;

template <typename S, bool DEV, int Q>
__global__ __launch_bounds__(kTotBlock) void k_totals_partial(Geom g, WallSpec w,
                                                              const S* __restrict__ f,
                                                              const S* __restrict__ psi,
                                                              double* __restrict__ part) {
  using L = Lat<Q>;
  __shared__ double red[10][kTotBlock];
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.N; s += gridDim.x * blockDim.x) {
    const int x = s % g.nx, y = (s / g.nx) % g.ny, z = s / (g.nx * g.ny);
    const Nbr nb(g, x, y, z);
    double r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double v = streamed_pop<S, Q>(g, w, f, nb, s, y, z, i);
      if (DEV) v += L::w[i] * w.rho0;
      r += v;
      if (L::cx[i]) jx += L::cx[i] * v;
      if (L::cy[i]) jy += L::cy[i] * v;
      if (L::cz[i]) jz += L::cz[i] * v;
    }
    const double p = static_cast<double>(psi[s]);
    acc[0] += r; acc[1] += jx; acc[2] += jy; acc[3] += jz; acc[4] += p;
    acc[5] += fabs(r); acc[6] += fabs(jx); acc[7] += fabs(jy); acc[8] += fabs(jz);
    acc[9] += fabs(p);
  }
#pragma unroll
  for (int k = 0; k < 10; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int w = kTotBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < 10; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 10) part[blockIdx.x * 10 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_totals_final(int nparts, const double* __restrict__ part,
                               double* __restrict__ out) {
  const int k = threadIdx.x;
  if (k >= 10) return;
  double acc = 0.0;
  for (int b = 0; b < nparts; ++b) acc += part[b * 10 + k];
  out[k] = acc;
}

}  // namespace lbl
