// lbl_kernels.hpp -- gfx950 kernels of the coupled FLBE + SMOL step.
//
// Storage type S is double (FP64 path) or float (FP32-deviation path, where
// populations hold fbar_i - w_i rho0).  Arithmetic runs in S.  One thread
// updates one site; neighbour values come through L1/L2.  Populations are
// structure-of-arrays: f[i*N + s].  The stored population buffer holds the
// post-collision values f*^{n-1}; step n pulls fbar^n(x) = f*^{n-1}(x - c_i).
#pragma once

#include "lbl_device.hpp"

namespace lbl {

enum : int { kFD = 0, kFV = 1 };

template <typename S>
struct Coef {
  S a, b, kappa, M;
};

// ---------------------------------------------------------------------------
// Chemical potential mu = A phi + B phi^3 - K L_SO phi  (Sec. II.A; the
// Shinozaki-Oono Laplacian of Eq. (solap) in 3-D, its 2-D analogue in 2-D).
// ---------------------------------------------------------------------------
template <typename S, int Q>
__device__ __forceinline__ S lap_so(const S* __restrict__ f, const Geom& g, int x, int y, int z) {
  S s1 = 0, s2 = 0, s3 = 0;
  if constexpr (Q == 19) {
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int r2 = dx * dx + dy * dy + dz * dz;
          if (r2 == 0) continue;
          const S v = f[g.nb(x, y, z, dx, dy, dz)];
          if (r2 == 1) s1 += v;
          else if (r2 == 2) s2 += v;
          else s3 += v;
        }
    return S(6.0 / 22.0) * s1 + S(3.0 / 22.0) * s2 + S(1.0 / 22.0) * s3 -
           S(80.0 / 22.0) * f[g.idx(x, y, z)];
  } else {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int r2 = dx * dx + dy * dy;
        if (r2 == 0) continue;
        const S v = f[g.nb(x, y, 0, dx, dy, 0)];
        if (r2 == 1) s1 += v;
        else s2 += v;
      }
    return S(0.5) * s1 + S(0.25) * s2 - S(3.0) * f[g.idx(x, y, 0)];
  }
}

template <typename S, int Q>
__global__ __launch_bounds__(256) void k_mu(Geom g, Coef<S> c, const S* __restrict__ phi,
                                            S* __restrict__ mu) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const int x = s % g.nx, y = (s / g.nx) % g.ny, z = s / (g.nx * g.ny);
  const S p = phi[s];
  mu[s] = c.a * p + c.b * p * p * p - c.kappa * lap_so<S, Q>(phi, g, x, y, z);
}

// Gradient of a scalar at (x,y,z): FD central difference (Sec. IV) or the FV
// Gamma operator (1/c_s^2) sum_i w_i c_i v(x + c_i)  (Eq. fvgrad).
template <typename S, int Q, int SMOL>
__device__ __forceinline__ void grad(const S* __restrict__ v, const Geom& g, int x, int y, int z,
                                     S out[3]) {
  using L = Lat<Q>;
  if constexpr (SMOL == kFD) {
    out[0] = S(0.5) * (v[g.nb(x, y, z, 1, 0, 0)] - v[g.nb(x, y, z, -1, 0, 0)]);
    out[1] = S(0.5) * (v[g.nb(x, y, z, 0, 1, 0)] - v[g.nb(x, y, z, 0, -1, 0)]);
    out[2] = L::D == 3 ? S(0.5) * (v[g.nb(x, y, z, 0, 0, 1)] - v[g.nb(x, y, z, 0, 0, -1)]) : S(0);
  } else {
    S gx = 0, gy = 0, gz = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const S t = S(L::w[i]) * v[g.nb(x, y, z, L::cx[i], L::cy[i], L::cz[i])];
      if (L::cx[i]) gx += L::cx[i] * t;
      if (L::cy[i]) gy += L::cy[i] * t;
      if (L::cz[i]) gz += L::cz[i] * t;
    }
    out[0] = S(3) * gx;
    out[1] = S(3) * gy;
    out[2] = S(3) * gz;
  }
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
  int noise;  // 0: kT == 0
  int collide;  // 0: only compute u (observe)
};

template <typename S, bool DEV, int Q, int SMOL>
__global__ __launch_bounds__(256) void k_lb(LBArgs<S> a) {
  using L = Lat<Q>;
  constexpr int D = L::D;
  constexpr int NR = Q - D - 1;
  constexpr int NB = (NR + 3) / 4;
  const Geom& g = a.g;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const int x = s % g.nx, y = (s / g.nx) % g.ny, z = s / (g.nx * g.ny);

  S F[3] = {0, 0, 0};
  if (a.force) {
    S gm[3];
    grad<S, Q, SMOL>(a.mu, g, x, y, z, gm);
    const S ps = a.psi[s];
    F[0] = -ps * gm[0];
    F[1] = -ps * gm[1];
    F[2] = -ps * gm[2];
  }

  S fv[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i)
    fv[i] = a.f_in[static_cast<size_t>(i) * g.N + g.nb(x, y, z, -L::cx[i], -L::cy[i], -L::cz[i])];

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
    a.u_out[s] = ux;
    a.u_out[g.N + s] = uy;
    if (D == 3) a.u_out[2 * g.N + s] = uz;
  }
  if (!a.collide) return;

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
  const S invD = S(1) / S(D);
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

  // Amplitudes n_k of the non-conserved modes k = D+1 .. Q-1: noise, plus the
  // surviving ghost part gamma_g m_g.
  constexpr auto& E = Modes<Q>::B.e;
  S nk[NB * 4];
#pragma unroll
  for (int k = 0; k < NB * 4; ++k) nk[k] = 0;
  if (a.noise) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      S z4[4];
      Normal4<S>::gen(static_cast<uint32_t>(s), a.step, b, kTagLB, a.k0, a.k1, z4);
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const int k = 4 * b + l;
        const S sig = k == 0 ? a.sigma_b : (k < L::NSTRESS ? a.sigma_s : a.sigma_g);
        nk[k] = sig * z4[l];
      }
    }
  }
  if (a.gamma_g != S(0)) {
#pragma unroll
    for (int k = L::NSTRESS; k < NR; ++k) {
      S m = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (E[D + 1 + k][i] != 0.0) m += S(E[D + 1 + k][i]) * fv[i];
      nk[k] += a.gamma_g * m;
    }
  }

#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = L::cx[i], cy = L::cy[i], cz = L::cz[i];
    S cj = 0;
    if (cx) cj += cx * jsx;
    if (cy) cj += cy * jsy;
    if (cz) cj += cz * jsz;
    S pq = -S(kCs2) * qtr;
    if (cx) pq += qxx;
    if (cy) pq += qyy;
    if (cz) pq += qzz;
    if (cx * cy) pq += S(2 * cx * cy) * qxy;
    if (cx * cz) pq += S(2 * cx * cz) * qxz;
    if (cy * cz) pq += S(2 * cy * cz) * qyz;
    S nz = 0;
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if (E[D + 1 + k][i] != 0.0) nz += S(E[D + 1 + k][i]) * nk[k];
    a.f_out[static_cast<size_t>(i) * g.N + s] = S(L::w[i]) * (S0 + S(3) * cj + S(4.5) * pq + nz);
  }
}

// ---------------------------------------------------------------------------
// SMOL noise term N^n, frozen over the Runge-Kutta stages (Sec. V).
// FD: link fluxes, N(x) = sum_l A_l [zeta_l(x - c_l) - zeta_l(x)],
//     A_l = sqrt(2 kT M lambda_l): the Gaussian law of Eq. (etafdt) built in
//     real space.  FV: N = Gamma . xi, xi_a = sqrt(2 kT M) z_a (Eqs. fvdiff,
//     noiseflux, fdt_orderpara).
// ---------------------------------------------------------------------------
template <typename S, int Q, int SMOL>
__global__ __launch_bounds__(256) void k_smol_noise(Geom g, S amp, uint32_t k0, uint32_t k1,
                                                    uint32_t step, S* __restrict__ out) {
  using L = Lat<Q>;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const int x = s % g.nx, y = (s / g.nx) % g.ny, z = s / (g.nx * g.ny);
  S acc = 0;
  if constexpr (SMOL == kFD) {
    constexpr int NL = L::NLINKS;
    constexpr int NB = (NL + 3) / 4;
    S own[NB * 4];
#pragma unroll
    for (int b = 0; b < NB; ++b) Normal4<S>::gen(s, step, b, kTagSMOL, k0, k1, own + 4 * b);
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int back = g.nb(x, y, z, -L::lx[l], -L::ly[l], -L::lz[l]);
      const S zb = normal_slot<S>(static_cast<uint32_t>(back), step, l, kTagSMOL, k0, k1);
      acc += amp * sqrt(S(L::lw[l])) * (zb - own[l]);
    }
  } else {
    S gx = 0, gy = 0, gz = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int t = g.nb(x, y, z, L::cx[i], L::cy[i], L::cz[i]);
      S xi[4];
      if constexpr (L::D == 2) {
        Normal4<S>::gen2(t, step, 0, kTagSMOL, k0, k1, xi);
      } else {
        Normal4<S>::gen(t, step, 0, kTagSMOL, k0, k1, xi);
      }
      if (L::cx[i]) gx += S(L::w[i] * L::cx[i]) * xi[0];
      if (L::cy[i]) gy += S(L::w[i] * L::cy[i]) * xi[1];
      if (L::D == 3 && L::cz[i]) gz += S(L::w[i] * L::cz[i]) * xi[2];
    }
    acc = S(3) * amp * (gx + gy + gz);
  }
  out[s] = acc;
}

// FV: g = Gamma mu on every site (needed at neighbours by the diffusion term).
template <typename S, int Q>
__global__ __launch_bounds__(256) void k_grad_fv(Geom g, const S* __restrict__ mu,
                                                 S* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const int x = s % g.nx, y = (s / g.nx) % g.ny, z = s / (g.nx * g.ny);
  S v[3];
  grad<S, Q, kFV>(mu, g, x, y, z, v);
  out[s] = v[0];
  out[g.N + s] = v[1];
  if (Lat<Q>::D == 3) out[2 * g.N + s] = v[2];
}

// ---------------------------------------------------------------------------
// One Runge-Kutta stage of SMOL with frozen u and N (Sec. V):
//   G(phi) = -Div(u phi) + M L_out mu(phi) + N,
// FD: Div central, L_out = L_SO.  FV: Div = Gamma., L_out mu = Gamma.(Gamma mu).
// Then  next = psi^n + cnext G,  acc = (first ? 0 : acc) + cacc G,
// and on the last stage out = psi^n + acc_prev + cacc G.
// ---------------------------------------------------------------------------
template <typename S>
struct StageArgs {
  Geom g;
  Coef<S> c;
  const S* phi;    // stage input
  const S* mu;     // mu(phi)
  const S* gmu;    // FV: Gamma mu(phi) (d*N)
  const S* u;      // u^n (d*N) or nullptr when const_u
  S u0, u1, u2;    // uniform imposed flow (SMOL_ONLY)
  const S* noise;  // N^n
  const S* psi_n;
  S* next;         // next stage input (or the new psi on the last stage)
  S* acc;
  S cnext, cacc;
  int first, last;
};

template <typename S, int Q, int SMOL>
__global__ __launch_bounds__(256) void k_smol_stage(StageArgs<S> a) {
  using L = Lat<Q>;
  const Geom& g = a.g;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const int x = s % g.nx, y = (s / g.nx) % g.ny, z = s / (g.nx * g.ny);
  const S* __restrict__ phi = a.phi;
  auto uval = [&](int comp, int t) -> S {
    if (a.u) return a.u[static_cast<size_t>(comp) * g.N + t];
    return comp == 0 ? a.u0 : (comp == 1 ? a.u1 : a.u2);
  };
  S adv = 0, lap = 0;
  if constexpr (SMOL == kFD) {
    const int xp = g.nb(x, y, z, 1, 0, 0), xm = g.nb(x, y, z, -1, 0, 0);
    const int yp = g.nb(x, y, z, 0, 1, 0), ym = g.nb(x, y, z, 0, -1, 0);
    adv = S(0.5) * (uval(0, xp) * phi[xp] - uval(0, xm) * phi[xm]) +
          S(0.5) * (uval(1, yp) * phi[yp] - uval(1, ym) * phi[ym]);
    if (L::D == 3) {
      const int zp = g.nb(x, y, z, 0, 0, 1), zm = g.nb(x, y, z, 0, 0, -1);
      adv += S(0.5) * (uval(2, zp) * phi[zp] - uval(2, zm) * phi[zm]);
    }
    lap = lap_so<S, Q>(a.mu, g, x, y, z);
  } else {
    S av = 0, dv = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int t = g.nb(x, y, z, L::cx[i], L::cy[i], L::cz[i]);
      const S p = phi[t];
      S ca = 0, cd = 0;
      if (L::cx[i]) { ca += L::cx[i] * uval(0, t); cd += L::cx[i] * a.gmu[t]; }
      if (L::cy[i]) { ca += L::cy[i] * uval(1, t); cd += L::cy[i] * a.gmu[g.N + t]; }
      if (L::cz[i]) { ca += L::cz[i] * uval(2, t); cd += L::cz[i] * a.gmu[2 * g.N + t]; }
      av += S(L::w[i]) * ca * p;
      dv += S(L::w[i]) * cd;
    }
    adv = S(3) * av;
    lap = S(3) * dv;
  }
  const S G = -adv + a.c.M * lap + a.noise[s];
  const S prev = a.first ? S(0) : a.acc[s];
  if (a.last) {
    a.next[s] = a.psi_n[s] + prev + a.cacc * G;
  } else {
    a.next[s] = a.psi_n[s] + a.cnext * G;
    a.acc[s] = prev + a.cacc * G;
  }
}

// ---------------------------------------------------------------------------
// Initial state and observables.
// ---------------------------------------------------------------------------
template <typename S, bool DEV, int Q>
__global__ __launch_bounds__(256) void k_init_uniform(Geom g, double rho0, double ux, double uy,
                                                      double uz, S* __restrict__ f) {
  using L = Lat<Q>;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const double usq = ux * ux + uy * uy + uz * uz;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double cu = L::cx[i] * ux + L::cy[i] * uy + L::cz[i] * uz;
    const double fe = L::w[i] * rho0 * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
    f[static_cast<size_t>(i) * g.N + s] = static_cast<S>(DEV ? fe - L::w[i] * rho0 : fe);
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

// Stored f*(x) = fbar(x + c_i) for a user fbar given in FP64.
template <typename S, bool DEV, int Q>
__global__ __launch_bounds__(256) void k_scatter_user(Geom g, double rho0,
                                                      const double* __restrict__ fin,
                                                      S* __restrict__ f) {
  using L = Lat<Q>;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const int x = s % g.nx, y = (s / g.nx) % g.ny, z = s / (g.nx * g.ny);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double v = fin[static_cast<size_t>(i) * g.N + g.nb(x, y, z, L::cx[i], L::cy[i], L::cz[i])];
    f[static_cast<size_t>(i) * g.N + s] = static_cast<S>(DEV ? v - L::w[i] * rho0 : v);
  }
}

// fbar(x) = f*(x - c_i), in FP64 (+ w_i rho0 for deviations); rho optional.
template <typename S, bool DEV, int Q>
__global__ __launch_bounds__(256) void k_gather(Geom g, double rho0, const S* __restrict__ f,
                                                double* __restrict__ pop,
                                                double* __restrict__ rho) {
  using L = Lat<Q>;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const int x = s % g.nx, y = (s / g.nx) % g.ny, z = s / (g.nx * g.ny);
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    double v = static_cast<double>(
        f[static_cast<size_t>(i) * g.N + g.nb(x, y, z, -L::cx[i], -L::cy[i], -L::cz[i])]);
    if (DEV) v += L::w[i] * rho0;
    if (pop) pop[static_cast<size_t>(i) * g.N + s] = v;
    r += v;
  }
  if (rho) rho[s] = r;
}

template <typename S>
__global__ __launch_bounds__(256) void k_to_f64(int n, const S* __restrict__ in,
                                                double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) out[s] = static_cast<double>(in[s]);
}

template <typename S>
__global__ __launch_bounds__(256) void k_from_f64(int n, const double* __restrict__ in,
                                                  S* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) out[s] = static_cast<S>(in[s]);
}

// Totals in FP64: per-block partials of (rho, j, psi, |rho|, |j|, |psi|),
// then one block sums the partials in a fixed order (deterministic).
constexpr int kTotBlock = 256;

template <typename S, bool DEV, int Q>
__global__ __launch_bounds__(kTotBlock) void k_totals_partial(Geom g, double rho0,
                                                              const S* __restrict__ f,
                                                              const S* __restrict__ psi,
                                                              double* __restrict__ part) {
  using L = Lat<Q>;
  __shared__ double red[10][kTotBlock];
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.N; s += gridDim.x * blockDim.x) {
    const int x = s % g.nx, y = (s / g.nx) % g.ny, z = s / (g.nx * g.ny);
    double r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double v = static_cast<double>(
          f[static_cast<size_t>(i) * g.N + g.nb(x, y, z, -L::cx[i], -L::cy[i], -L::cz[i])]);
      if (DEV) v += L::w[i] * rho0;
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
