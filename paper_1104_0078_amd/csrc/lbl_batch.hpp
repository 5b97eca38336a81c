// lbl_batch.hpp -- batched launches: many independent replicas of one kind
// (storage, lattice, variant) advance together.  Each launch walks a work
// table of (replica, block) items; the replica's buffers and parameters come
// from a descriptor array and its step counter and buffer parity from a
// device-side state array, so a graph can capture any number of steps.  The
// per-block arithmetic is the same device code as the single-simulation
// kernels (lb_body, prep_*_body, stage_*_body).
#pragma once

#include "lbl_kernels.hpp"

namespace lbl {

enum : int { kCplFull = 0, kCplSmolOnly = 1, kCplLbOnly = 2 };

template <typename S>
struct Replica {
  Geom g;
  Coef<S> c;
  int zc;
  int coupling;
  int noise_on;  // kT > 0
  S* f[2];
  S* psi[2];
  S* phi[2];
  S* acc;
  S* mu;
  S* u;
  S* u_end;
  S* noise;
  S rho0, gamma_s, gamma_b, gamma_g, sigma_s, sigma_b, sigma_g, amp;
  S u0, u1, u2;
  S uw[2][3];  // walls: velocities of the lower and upper wall
  uint32_t k0, k1;
};

// Device-side state of one replica at the start of a tick; it is advanced
// while remaining > 0.
struct RepState {
  int cur;    // population buffer holding f*
  int pcur;   // psi buffer holding psi^n
  uint32_t step;
  int remaining;
};

// The state k steps into a tick: the buffers flip every step (those the
// coupling updates), the counters move by k.  The launches of step k of a
// captured tick take k as an argument, so no kernel has to advance the state
// between steps; kb_advance moves it once, at the end of the tick.
__device__ __forceinline__ RepState at_step(RepState s, int coupling, int k) {
  if (coupling != kCplSmolOnly && (k & 1)) s.cur = 1 - s.cur;
  if (coupling != kCplLbOnly && (k & 1)) s.pcur = 1 - s.pcur;
  s.step += static_cast<uint32_t>(k);
  s.remaining -= k;
  return s;
}

struct Work {
  int rep;
  int bx, by, bz;
};

// WALLS: every replica of the launch has walls across the last axis (FV).
template <typename S, int Q, int SMOL, bool WALLS = false>
__global__ __launch_bounds__(kTX* kTY) void kb_prep(const Replica<S>* __restrict__ reps,
                                                   const RepState* __restrict__ st,
                                                   const Work* __restrict__ work, int k) {
  const Work w = work[blockIdx.x];
  const Replica<S>& r = reps[w.rep];
  const RepState rs = at_step(st[w.rep], r.coupling, k);
  if (rs.remaining <= 0) return;
  PrepArgs<S> a;
  a.g = r.g;
  a.c = r.c;
  a.amp = r.amp;
  a.k0 = r.k0;
  a.k1 = r.k1;
  a.step = rs.step;
  a.zc = r.zc;
  a.psi = r.psi[rs.pcur];
  // the SMOL noise is drawn in kb_uend_noise; the preparation computes mu
  a.noise = nullptr;
  a.mu = r.coupling == kCplFull ? r.mu : nullptr;
  if (!a.mu) return;
  if constexpr (SMOL == kFV)
    prep_fv_body<S, Q, WALLS>(a, w.bx, w.by, w.bz);
  else
    prep_fd_body<S, Q>(a, w.bx, w.by, w.bz);
}

// LB work items are tiles of 2^lw sites along x by 256 / 2^lw rows of one
// plane (one 256-thread block each).
__device__ __forceinline__ void lb_tile_site(const Work& w, int lw, int& x, int& y) {
  x = (w.bx << lw) + (threadIdx.x & ((1 << lw) - 1));
  y = w.by * (kSiteBlock >> lw) + (threadIdx.x >> lw);
}

template <typename S, bool DEV, int Q, int SMOL, bool GHOST, bool NT, bool WALLS = false>
__global__ __launch_bounds__(kSiteBlock) void kb_lb(const Replica<S>* __restrict__ reps,
                                                      const RepState* __restrict__ st,
                                                      const Work* __restrict__ work, int lw,
                                                      int k) {
  const Work w = work[blockIdx.x];
  const Replica<S>& r = reps[w.rep];
  const RepState rs = at_step(st[w.rep], r.coupling, k);
  if (rs.remaining <= 0 || r.coupling == kCplSmolOnly) return;
  LBArgs<S> a;
  a.g = r.g;
  a.f_in = r.f[rs.cur];
  a.f_out = r.f[1 - rs.cur];
  a.psi = r.psi[rs.pcur];
  a.mu = r.mu;
  a.u_out = r.u;
  a.rho0 = r.rho0;
  a.gamma_s = r.gamma_s;
  a.gamma_b = r.gamma_b;
  a.gamma_g = r.gamma_g;
  a.sigma_s = r.sigma_s;
  a.sigma_b = r.sigma_b;
  a.sigma_g = r.sigma_g;
  a.k0 = r.k0;
  a.k1 = r.k1;
  a.step = rs.step;
  a.force = r.coupling == kCplFull;
  a.Fext = nullptr;
  a.noise = r.noise_on;
  a.nt = NT;
  for (int k = 0; k < 2; ++k)
    for (int c = 0; c < 3; ++c) a.uw[k][c] = r.uw[k][c];
  int x, y;
  lb_tile_site(w, lw, x, y);
  if (x < r.g.nx && y < r.g.ny) lb_body<S, DEV, Q, SMOL, GHOST, true, NT, WALLS>(a, x, y, w.bz);
}

// The velocity of the streamed populations, (jbar^{n+1} + F^n/2)/rho^{n+1},
// for the Runge-Kutta stages at t_{n+1} (full coupling, rk >= 2: the LB body
// without collision, pulling the populations the step just wrote), and the
// SMOL noise (kT > 0, a coupling with the SMOL update) in one launch over the
// SMOL tiles, as k_uend_noise; each replica does the parts it needs.
template <typename S, bool DEV, int Q, int SMOL, bool NT, bool WALLS = false>
__global__ __launch_bounds__(kTX* kTY) void kb_uend_noise(const Replica<S>* __restrict__ reps,
                                                         const RepState* __restrict__ st,
                                                         const Work* __restrict__ work, int rk,
                                                         int k) {
  const Work w = work[blockIdx.x];
  const Replica<S>& r = reps[w.rep];
  const RepState rs = at_step(st[w.rep], r.coupling, k);
  if (rs.remaining <= 0) return;
  const bool pull = r.coupling == kCplFull && rk >= 2;
  const bool noise = r.coupling != kCplLbOnly && r.noise_on;
  if (!pull && !noise) return;
  LBArgs<S> la;
  la.g = r.g;
  la.f_in = r.f[1 - rs.cur];
  la.f_out = nullptr;
  la.psi = r.psi[rs.pcur];
  la.mu = r.mu;
  la.u_out = r.u_end;
  la.rho0 = r.rho0;
  la.force = 1;
  la.Fext = nullptr;
  la.noise = 0;
  la.nt = NT;
  for (int c = 0; c < 2; ++c)
    for (int d = 0; d < 3; ++d) la.uw[c][d] = r.uw[c][d];
  PrepArgs<S> pa;
  pa.g = r.g;
  pa.c = r.c;
  pa.amp = r.amp;
  pa.k0 = r.k0;
  pa.k1 = r.k1;
  pa.step = rs.step;
  pa.zc = r.zc;
  pa.psi = nullptr;
  pa.noise = noise ? r.noise : nullptr;
  pa.mu = nullptr;
  uend_noise_body<S, DEV, Q, SMOL, NT, WALLS>(la, pa, pull, w.bx, w.by, w.bz);
}

// Stage `st` of `ns` (ns = 1, 2 or 4), with the same combinations as the
// single-simulation path.
template <typename S, int Q, int SMOL, bool WALLS = false>
__global__ __launch_bounds__(kTX* kTY) void kb_stage(const Replica<S>* __restrict__ reps,
                                                    const RepState* __restrict__ state,
                                                    const Work* __restrict__ work, int st,
                                                    int ns, int k) {
  const Work w = work[blockIdx.x];
  const Replica<S>& r = reps[w.rep];
  const RepState rs = at_step(state[w.rep], r.coupling, k);
  if (rs.remaining <= 0 || r.coupling == kCplLbOnly) return;
  StageArgs<S> a;
  a.g = r.g;
  a.c = r.c;
  a.phi = st == 0 ? r.psi[rs.pcur] : r.phi[(st - 1) & 1];
  a.u = r.coupling == kCplFull ? r.u : nullptr;
  a.u_end = r.u_end;
  a.utime = st == 0 ? kAtN : (st == ns - 1 ? kAtN1 : kAtMid);
  a.u0 = r.u0;
  a.u1 = r.u1;
  a.u2 = r.u2;
  a.noise = r.noise;
  a.psi_n = r.psi[rs.pcur];
  a.first = st == 0;
  a.last = st == ns - 1;
  a.zc = r.zc;
  a.acc = nullptr;
  a.cacc = S(0);
  a.cnext = S(1);
  a.mode = kComb;
  if (ns == 2 && st == 1) a.mode = kHeun2;
  if (ns == 4) {
    a.acc = r.acc;
    a.cnext = st == 2 ? S(1) : S(0.5);
    a.cacc = (st == 0 || st == 3) ? S(1.0 / 6.0) : S(1.0 / 3.0);
  }
  a.out = a.last ? r.psi[1 - rs.pcur] : r.phi[st & 1];
  if constexpr (SMOL == kFV)
    stage_fv_body<S, Q, WALLS>(a, w.bx, w.by, w.bz);
  else
    stage_fd_body<S, Q>(a, w.bx, w.by, w.bz);
}

// End of a tick of `nsteps` steps: each replica's state after the steps it
// took (up to its own count).
template <typename S>
__global__ void kb_advance(const Replica<S>* __restrict__ reps, RepState* __restrict__ st, int n,
                           int nsteps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const RepState s = st[i];
  if (s.remaining <= 0) return;
  st[i] = at_step(s, reps[i].coupling, s.remaining < nsteps ? s.remaining : nsteps);
}

}  // namespace lbl
