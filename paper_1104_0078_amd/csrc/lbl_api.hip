// lbl_api.hip -- the C ABI of include/lbl.h: simulation lifecycle, parameter
// validation, device memory through the injected allocator, and the per-step
// launch sequence of the coupled FLBE + SMOL sweep.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "lbl.h"
#include "lbl_kernels.hpp"

using namespace lbl;

namespace {

thread_local std::string g_create_error;

constexpr int kBlock = 256;

}  // namespace

struct lbl_sim {
  lbl_params p{};
  int q = 0, d = 0, N = 0, Lmax = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  lbl_alloc_fn alloc = nullptr;
  lbl_free_fn free_fn = nullptr;
  void* ctx = nullptr;
  size_t ssize = 8;  // bytes per stored value
  std::vector<void*> owned;
  void* f[2] = {nullptr, nullptr};
  int cur = 0;
  void* psi[2] = {nullptr, nullptr};
  int pcur = 0;
  void* phi[2] = {nullptr, nullptr};
  void* acc = nullptr;
  void* mu = nullptr;
  void* u = nullptr;
  void* noise = nullptr;
  double* part = nullptr;
  int nparts = 0;
  double* tot = nullptr;
  int64_t step = 0;
  int64_t nsamples = 0;
  uint32_t k0 = 0, k1 = 0;
  int zc = 1;  // planes per block of the z-marching kernels
  double gamma_s = 0, gamma_b = 0, gamma_g = 0, sigma_s = 0, sigma_b = 0, sigma_g = 0;
  int deferred = LBL_OK;
  std::string err;
  // Event timing of step kernels.
  bool timing = false;
  struct Pending {
    int slot;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  std::vector<lbl_kernel_time> kt;
};

namespace {

int fail(lbl_sim* s, int code, const std::string& msg) {
  if (s)
    s->err = msg;
  else
    g_create_error = msg;
  return code;
}

int hip_check(lbl_sim* s, hipError_t e, const char* what) {
  if (e == hipSuccess) return LBL_OK;
  return fail(s, LBL_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void* dev_alloc(lbl_sim* s, size_t bytes) {
  void* ptr = nullptr;
  if (bytes == 0) bytes = 8;
  if (s->alloc) {
    ptr = s->alloc(s->ctx, bytes, s->stream);
  } else if (hipMalloc(&ptr, bytes) != hipSuccess) {
    ptr = nullptr;
  }
  if (ptr) s->owned.push_back(ptr);
  return ptr;
}

void dev_free(lbl_sim* s, void* ptr) {
  if (!ptr) return;
  if (s->free_fn)
    s->free_fn(s->ctx, ptr, s->stream);
  else
    (void)hipFree(ptr);
}

// Free one allocation made by dev_alloc before the simulation ends.
void dev_release(lbl_sim* s, void* ptr) {
  if (!ptr) return;
  (void)hipStreamSynchronize(s->stream);
  for (size_t k = 0; k < s->owned.size(); ++k)
    if (s->owned[k] == ptr) {
      s->owned.erase(s->owned.begin() + static_cast<long>(k));
      break;
    }
  dev_free(s, ptr);
}

void release_all(lbl_sim* s) {
  if (!s) return;
  if (!s->owned.empty()) (void)hipStreamSynchronize(s->stream);
  for (void* ptr : s->owned) dev_free(s, ptr);
  s->owned.clear();
}

inline int grid_for(int n) { return (n + kBlock - 1) / kBlock; }

hipEvent_t take_event(lbl_sim* s) {
  if (!s->event_pool.empty()) {
    hipEvent_t e = s->event_pool.back();
    s->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int kernel_slot(lbl_sim* s, const char* name) {
  for (size_t k = 0; k < s->kt.size(); ++k)
    if (std::strncmp(s->kt[k].name, name, sizeof(s->kt[k].name)) == 0) return static_cast<int>(k);
  lbl_kernel_time t{};
  std::strncpy(t.name, name, sizeof(t.name) - 1);
  s->kt.push_back(t);
  return static_cast<int>(s->kt.size()) - 1;
}

// Launch `fn` (a kernel launch on s->stream), bracketed by timing events when
// timing is enabled, and check the launch.
template <class Fn>
int launch(lbl_sim* s, const char* name, Fn&& fn) {
  hipEvent_t a = nullptr, b = nullptr;
  if (s->timing) {
    a = take_event(s);
    b = take_event(s);
    if (a) (void)hipEventRecord(a, s->stream);
  }
  fn();
  const hipError_t e = hipGetLastError();
  if (s->timing && a && b) {
    (void)hipEventRecord(b, s->stream);
    s->pending.push_back(lbl_sim::Pending{kernel_slot(s, name), a, b});
  }
  return hip_check(s, e, name);
}

int drain_timing(lbl_sim* s) {
  if (s->pending.empty()) return LBL_OK;
  if (int rc = hip_check(s, hipStreamSynchronize(s->stream), "timing sync")) return rc;
  for (auto& p : s->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      s->kt[p.slot].total_ms += ms;
      s->kt[p.slot].launches += 1;
    }
    s->event_pool.push_back(p.a);
    s->event_pool.push_back(p.b);
  }
  s->pending.clear();
  return LBL_OK;
}

void destroy_events(lbl_sim* s) {
  for (auto& p : s->pending) {
    s->event_pool.push_back(p.a);
    s->event_pool.push_back(p.b);
  }
  s->pending.clear();
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  s->event_pool.clear();
}

bool finite_all(const lbl_params& p) {
  const double v[] = {p.rho, p.eta, p.M, p.a, p.b, p.kappa, p.kT, p.omega_bulk, p.omega_ghost,
                      p.u_imposed[0], p.u_imposed[1], p.u_imposed[2]};
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

int validate(const lbl_params* p, const lbl_init* in) {
  if (!p || !in) return fail(nullptr, LBL_E_INVAL, "params and init must not be NULL");
  if (p->lattice != LBL_D2Q9 && p->lattice != LBL_D3Q19)
    return fail(nullptr, LBL_E_INVAL, "lattice must be LBL_D2Q9 or LBL_D3Q19");
  if (p->smol != LBL_SMOL_FD && p->smol != LBL_SMOL_FV)
    return fail(nullptr, LBL_E_INVAL, "smol must be LBL_SMOL_FD or LBL_SMOL_FV");
  if (p->precision != LBL_FP64 && p->precision != LBL_FP32DEV)
    return fail(nullptr, LBL_E_INVAL, "precision must be LBL_FP64 or LBL_FP32DEV");
  if (p->coupling < LBL_FULL || p->coupling > LBL_LB_ONLY)
    return fail(nullptr, LBL_E_INVAL, "unknown coupling");
  if (p->rk_stages != 1 && p->rk_stages != 2 && p->rk_stages != 4)
    return fail(nullptr, LBL_E_INVAL, "rk_stages must be 1, 2 or 4");
  if (p->nx < 4 || p->ny < 4) return fail(nullptr, LBL_E_INVAL, "nx and ny must be >= 4");
  if (p->lattice == LBL_D2Q9 && p->nz != 1) return fail(nullptr, LBL_E_INVAL, "D2Q9 needs nz == 1");
  if (p->lattice == LBL_D3Q19 && p->nz < 4) return fail(nullptr, LBL_E_INVAL, "nz must be >= 4");
  const double n = static_cast<double>(p->nx) * p->ny * p->nz;
  if (n >= 2147483648.0) return fail(nullptr, LBL_E_INVAL, "nx*ny*nz must be < 2^31");
  if (!finite_all(*p)) return fail(nullptr, LBL_E_INVAL, "parameters must be finite");
  if (!(p->rho > 0)) return fail(nullptr, LBL_E_INVAL, "rho must be > 0");
  if (!(p->eta > 0)) return fail(nullptr, LBL_E_INVAL, "eta must be > 0");
  if (!(p->M >= 0)) return fail(nullptr, LBL_E_INVAL, "M must be >= 0");
  if (!(p->kT >= 0)) return fail(nullptr, LBL_E_INVAL, "kT must be >= 0");
  const double ws = 1.0 / (0.5 + p->eta / (p->rho * kCs2));
  if (!(ws > 0 && ws < 2)) return fail(nullptr, LBL_E_INVAL, "shear rate outside (0, 2)");
  if (!(p->omega_bulk > 0 && p->omega_bulk <= 2) || !(p->omega_ghost > 0 && p->omega_ghost <= 2))
    return fail(nullptr, LBL_E_INVAL, "omega_bulk and omega_ghost must lie in (0, 2]");
  if (p->sample_every < 0 || p->reserved != 0)
    return fail(nullptr, LBL_E_INVAL, "sample_every must be >= 0 and reserved 0");
  if (in->kind < LBL_INIT_REST || in->kind > LBL_INIT_USER)
    return fail(nullptr, LBL_E_INVAL, "unknown init kind");
  if (in->kind == LBL_INIT_TANH_2IF && !(p->a < 0 && p->b > 0 && p->kappa > 0))
    return fail(nullptr, LBL_E_INVAL, "two-phase init needs a < 0 < b and kappa > 0");
  if (in->kind == LBL_INIT_USER && (!in->psi0 || !in->f0))
    return fail(nullptr, LBL_E_INVAL, "USER init needs psi0 and f0");
  if (!std::isfinite(in->psi_std) || in->psi_std < 0)
    return fail(nullptr, LBL_E_INVAL, "psi_std must be finite and >= 0");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(in->boost_u[k])) return fail(nullptr, LBL_E_INVAL, "boost must be finite");
  return LBL_OK;
}

// ---------------------------------------------------------------------------
// Typed implementation for one (storage, lattice, variant) combination.
// ---------------------------------------------------------------------------
template <typename S, bool DEV, int Q, int SMOL>
struct Impl {
  static Geom geom(const lbl_sim* s) { return Geom{s->p.nx, s->p.ny, s->p.nz, s->N}; }
  static Coef<S> coef(const lbl_sim* s) {
    return Coef<S>{S(s->p.a), S(s->p.b), S(s->p.kappa), S(s->p.M)};
  }

  static int launched(lbl_sim* s, const char* what) {
    return hip_check(s, hipGetLastError(), what);
  }

  static int init(lbl_sim* s, const lbl_init* in) {
    const Geom g = geom(s);
    const int grid = grid_for(s->N);
    S* f = static_cast<S*>(s->f[0]);
    S* psi = static_cast<S*>(s->psi[0]);
    if (in->kind == LBL_INIT_USER) {
      const double* f0 = in->f0;
      const double* p0 = in->psi0;
      double* tmp = nullptr;
      const size_t fbytes = sizeof(double) * static_cast<size_t>(s->q) * s->N;
      const size_t pbytes = sizeof(double) * static_cast<size_t>(s->N);
      if (!in->user_on_device) {
        tmp = static_cast<double*>(dev_alloc(s, fbytes + pbytes));
        if (!tmp) return fail(s, LBL_E_NOMEM, "device allocation failed (user init staging)");
        int rc = hip_check(s, hipMemcpyAsync(tmp, f0, fbytes, hipMemcpyHostToDevice, s->stream),
                           "copy f0");
        if (rc) return rc;
        rc = hip_check(s, hipMemcpyAsync(tmp + static_cast<size_t>(s->q) * s->N, p0, pbytes,
                                         hipMemcpyHostToDevice, s->stream),
                       "copy psi0");
        if (rc) return rc;
        f0 = tmp;
        p0 = tmp + static_cast<size_t>(s->q) * s->N;
      }
      k_scatter_user<S, DEV, Q><<<grid, kBlock, 0, s->stream>>>(g, s->p.rho, f0, f);
      if (int rc = launched(s, "k_scatter_user")) return rc;
      k_from_f64<S><<<grid, kBlock, 0, s->stream>>>(s->N, p0, psi);
      if (int rc = launched(s, "k_from_f64")) return rc;
      if (tmp) {
        int rc = hip_check(s, hipStreamSynchronize(s->stream), "user init sync");
        dev_release(s, tmp);
        if (rc) return rc;
      }
      return LBL_OK;
    }
    k_init_uniform<S, DEV, Q><<<grid, kBlock, 0, s->stream>>>(
        g, s->p.rho, in->boost_u[0], in->boost_u[1], Lat<Q>::D == 3 ? in->boost_u[2] : 0.0, f);
    if (int rc = launched(s, "k_init_uniform")) return rc;
    double psi_eq = 0, l = 1;
    const int tanh_on = in->kind == LBL_INIT_TANH_2IF;
    if (tanh_on) {
      psi_eq = std::sqrt(-s->p.a / s->p.b);
      l = std::sqrt(-2.0 * s->p.kappa / s->p.a);
    }
    k_init_psi<S, Q><<<grid, kBlock, 0, s->stream>>>(g, in->psi_std, tanh_on, psi_eq, l, s->k0,
                                                     s->k1, psi);
    return launched(s, "k_init_psi");
  }

  static LBArgs<S> lb_args(lbl_sim* s, const S* fin, S* fout, const S* psi, S* u_out,
                           int force, uint32_t step) {
    LBArgs<S> a;
    a.g = geom(s);
    a.f_in = fin;
    a.f_out = fout;
    a.psi = psi;
    a.mu = static_cast<const S*>(s->mu);
    a.u_out = u_out;
    a.rho0 = S(s->p.rho);
    a.gamma_s = S(s->gamma_s);
    a.gamma_b = S(s->gamma_b);
    a.gamma_g = S(s->gamma_g);
    a.sigma_s = S(s->sigma_s);
    a.sigma_b = S(s->sigma_b);
    a.sigma_g = S(s->sigma_g);
    a.k0 = s->k0;
    a.k1 = s->k1;
    a.step = step;
    a.force = force;
    a.noise = s->p.kT > 0;
    return a;
  }

  static dim3 site_grid(const lbl_sim* s) {
    return dim3((s->p.nx + kBX - 1) / kBX, (s->p.ny + kBY - 1) / kBY, s->p.nz);
  }
  static dim3 tile_grid(const lbl_sim* s) {
    return dim3((s->p.nx + kTX - 1) / kTX, (s->p.ny + kTY - 1) / kTY,
                Lat<Q>::D == 3 ? (s->p.nz + s->zc - 1) / s->zc : 1);
  }

  static int launch_lb(lbl_sim* s, const LBArgs<S>& a, bool collide) {
    const dim3 grid = site_grid(s), block(kBX, kBY);
    const bool ghost = s->gamma_g != 0.0;
    if (!collide)
      return launch(s, "k_lb_u", [&] {
        k_lb<S, DEV, Q, SMOL, false, false><<<grid, block, 0, s->stream>>>(a);
      });
    if (ghost)
      return launch(s, "k_lb", [&] {
        k_lb<S, DEV, Q, SMOL, true, true><<<grid, block, 0, s->stream>>>(a);
      });
    return launch(s, "k_lb", [&] {
      k_lb<S, DEV, Q, SMOL, false, true><<<grid, block, 0, s->stream>>>(a);
    });
  }

  static int launch_mu(lbl_sim* s, const S* phi, S* mu) {
    const dim3 grid = site_grid(s), block(kBX, kBY);
    const Geom g = geom(s);
    const Coef<S> c = coef(s);
    return launch(s, "k_mu", [&] { k_mu<S, Q><<<grid, block, 0, s->stream>>>(g, c, phi, mu); });
  }

  static int one_step(lbl_sim* s) {
    const Geom g = geom(s);
    const uint32_t n = static_cast<uint32_t>(s->step);
    const int cpl = s->p.coupling;
    S* fin = static_cast<S*>(s->f[s->cur]);
    S* fout = static_cast<S*>(s->f[1 - s->cur]);
    S* psin = static_cast<S*>(s->psi[s->pcur]);
    S* psout = static_cast<S*>(s->psi[1 - s->pcur]);
    S* u = static_cast<S*>(s->u);

    S* noise = static_cast<S*>(s->noise);
    const dim3 tg = tile_grid(s), tb(kTX, kTY);
    const bool want_noise = cpl != LBL_LB_ONLY && s->p.kT > 0;
    const bool want_mu = cpl == LBL_FULL;
    if (want_noise || want_mu) {
      PrepArgs<S> pa;
      pa.g = g;
      pa.c = coef(s);
      pa.amp = S(std::sqrt(2.0 * s->p.kT * s->p.M));
      pa.k0 = s->k0;
      pa.k1 = s->k1;
      pa.step = n;
      pa.zc = s->zc;
      pa.psi = psin;
      pa.noise = want_noise ? noise : nullptr;
      pa.mu = want_mu ? static_cast<S*>(s->mu) : nullptr;
      int rc;
      if (SMOL == kFV)
        rc = launch(s, "k_prep", [&] { k_prep_fv<S, Q><<<tg, tb, 0, s->stream>>>(pa); });
      else
        rc = launch(s, "k_prep", [&] { k_prep_fd<S, Q><<<tg, tb, 0, s->stream>>>(pa); });
      if (rc) return rc;
    }
    if (cpl != LBL_SMOL_ONLY) {
      const LBArgs<S> a = lb_args(s, fin, fout, psin, cpl == LBL_FULL ? u : nullptr,
                                  cpl == LBL_FULL, n);
      if (int rc = launch_lb(s, a, true)) return rc;
    }
    if (cpl != LBL_LB_ONLY) {
      const int ns = s->p.rk_stages;
      static const double cn4[4] = {0.5, 0.5, 1.0, 0.0};
      static const double ca4[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
      const S* phi = psin;
      for (int st = 0; st < ns; ++st) {
        StageArgs<S> a;
        a.g = g;
        a.c = coef(s);
        a.phi = phi;
        a.u = cpl == LBL_FULL ? u : nullptr;
        a.u0 = S(s->p.u_imposed[0]);
        a.u1 = S(s->p.u_imposed[1]);
        a.u2 = S(Lat<Q>::D == 3 ? s->p.u_imposed[2] : 0.0);
        a.noise = noise;
        a.psi_n = psin;
        a.first = st == 0;
        a.last = st == ns - 1;
        a.zc = s->zc;
        a.acc = nullptr;
        a.cacc = S(0);
        a.cnext = S(1);
        a.mode = kComb;
        if (ns == 2 && st == 1) a.mode = kHeun2;
        if (ns == 4) {
          a.acc = static_cast<S*>(s->acc);
          a.cnext = S(cn4[st]);
          a.cacc = S(ca4[st]);
        }
        a.out = a.last ? psout : static_cast<S*>(s->phi[st & 1]);
        int rc;
        if (SMOL == kFV)
          rc = launch(s, "k_stage",
                      [&] { k_stage_fv<S, Q><<<tg, tb, 0, s->stream>>>(a); });
        else
          rc = launch(s, "k_stage",
                      [&] { k_stage_fd<S, Q><<<tg, tb, 0, s->stream>>>(a); });
        if (rc) return rc;
        phi = a.out;
      }
      s->pcur = 1 - s->pcur;
    }
    if (cpl != LBL_SMOL_ONLY) s->cur = 1 - s->cur;
    s->step += 1;
    return LBL_OK;
  }

  static int steps(lbl_sim* s, int64_t nsteps) {
    for (int64_t k = 0; k < nsteps; ++k)
      if (int rc = one_step(s)) return rc;
    return LBL_OK;
  }

  // Observables into a device FP64 buffer `dst`.
  static int observe(lbl_sim* s, int what, double* dst) {
    const Geom g = geom(s);
    const int grid = grid_for(s->N);
    const S* f = static_cast<const S*>(s->f[s->cur]);
    const S* psi = static_cast<const S*>(s->psi[s->pcur]);
    switch (what) {
      case LBL_OBS_PSI:
        k_to_f64<S><<<grid, kBlock, 0, s->stream>>>(s->N, psi, dst);
        return launched(s, "k_to_f64");
      case LBL_OBS_POP:
        k_gather<S, DEV, Q><<<grid, kBlock, 0, s->stream>>>(g, s->p.rho, f, dst, nullptr);
        return launched(s, "k_gather");
      case LBL_OBS_RHO:
        k_gather<S, DEV, Q><<<grid, kBlock, 0, s->stream>>>(g, s->p.rho, f, nullptr, dst);
        return launched(s, "k_gather");
      case LBL_OBS_U: {
        if (s->p.coupling == LBL_SMOL_ONLY) return LBL_E_UNSUPPORTED;
        S* ubuf = static_cast<S*>(s->u);
        const int full = s->p.coupling == LBL_FULL;
        if (full)
          if (int rc = launch_mu(s, psi, static_cast<S*>(s->mu))) return rc;
        const LBArgs<S> a = lb_args(s, f, nullptr, psi, ubuf, full, 0);
        if (int rc = launch_lb(s, a, false)) return rc;
        k_to_f64<S><<<grid_for(s->d * s->N), kBlock, 0, s->stream>>>(s->d * s->N, ubuf, dst);
        return launched(s, "k_to_f64");
      }
      case LBL_OBS_TOTALS: {
        k_totals_partial<S, DEV, Q><<<s->nparts, kTotBlock, 0, s->stream>>>(g, s->p.rho, f, psi,
                                                                           s->part);
        if (int rc = launched(s, "k_totals_partial")) return rc;
        k_totals_final<<<1, 64, 0, s->stream>>>(s->nparts, s->part, dst);
        return launched(s, "k_totals_final");
      }
      default:
        return LBL_E_UNSUPPORTED;
    }
  }
};

using StepFn = int (*)(lbl_sim*, int64_t);
using InitFn = int (*)(lbl_sim*, const lbl_init*);
using ObsFn = int (*)(lbl_sim*, int, double*);

struct Table {
  StepFn step;
  InitFn init;
  ObsFn observe;
};

template <typename S, bool DEV, int Q, int SMOL>
Table table_for() {
  return Table{&Impl<S, DEV, Q, SMOL>::steps, &Impl<S, DEV, Q, SMOL>::init,
               &Impl<S, DEV, Q, SMOL>::observe};
}

Table select(const lbl_params& p) {
  const bool f32 = p.precision == LBL_FP32DEV;
  const bool d3 = p.lattice == LBL_D3Q19;
  const bool fv = p.smol == LBL_SMOL_FV;
  if (!f32) {
    if (!d3) return fv ? table_for<double, false, 9, kFV>() : table_for<double, false, 9, kFD>();
    return fv ? table_for<double, false, 19, kFV>() : table_for<double, false, 19, kFD>();
  }
  if (!d3) return fv ? table_for<float, true, 9, kFV>() : table_for<float, true, 9, kFD>();
  return fv ? table_for<float, true, 19, kFV>() : table_for<float, true, 19, kFD>();
}

size_t obs_bytes(const lbl_sim* s, int what) {
  const size_t N = static_cast<size_t>(s->N);
  switch (what) {
    case LBL_OBS_PSI:
    case LBL_OBS_RHO:
      return 8 * N;
    case LBL_OBS_U:
      return 8 * N * s->d;
    case LBL_OBS_POP:
      return 8 * N * s->q;
    case LBL_OBS_TOTALS:
      return 8 * 10;
    case LBL_OBS_SK_AXES:
      return 8 * static_cast<size_t>(s->d) * s->Lmax;
    case LBL_OBS_UK_AXES:
      return 8 * static_cast<size_t>(s->d) * s->d * s->Lmax;
    case LBL_OBS_STEP:
    case LBL_OBS_NSAMPLES:
      return 8;
    default:
      return 0;
  }
}

int create_impl(const lbl_params* params, const lbl_init* init, const lbl_env* env,
                lbl_sim** out) {
  if (!out) return fail(nullptr, LBL_E_INVAL, "out must not be NULL");
  *out = nullptr;
  if (int rc = validate(params, init)) return rc;
  lbl_sim* s = new (std::nothrow) lbl_sim();
  if (!s) return fail(nullptr, LBL_E_NOMEM, "host allocation failed");
  s->p = *params;
  s->q = params->lattice;
  s->d = params->lattice == LBL_D2Q9 ? 2 : 3;
  s->N = params->nx * params->ny * params->nz;
  s->Lmax = std::max(params->nx, std::max(params->ny, params->nz));
  s->ssize = params->precision == LBL_FP64 ? 8 : 4;
  s->k0 = static_cast<uint32_t>(params->seed);
  s->k1 = static_cast<uint32_t>(params->seed >> 32);
  if (env) {
    s->device = env->device;
    s->stream = static_cast<hipStream_t>(env->stream);
    s->alloc = env->alloc;
    s->free_fn = env->free;
    s->ctx = env->ctx;
  }
  if ((s->alloc == nullptr) != (s->free_fn == nullptr)) {
    delete s;
    return fail(nullptr, LBL_E_INVAL, "alloc and free must both be set or both NULL");
  }
  int rc = hip_check(nullptr, hipSetDevice(s->device), "hipSetDevice");
  if (rc) {
    g_create_error = s->err.empty() ? g_create_error : s->err;
    delete s;
    return rc;
  }
  // Relaxation rates and noise amplitudes of the mode classes.
  const double ws = 1.0 / (0.5 + params->eta / (params->rho * kCs2));
  s->gamma_s = 1.0 - ws;
  s->gamma_b = 1.0 - params->omega_bulk;
  s->gamma_g = 1.0 - params->omega_ghost;
  auto sig = [&](double g) { return std::sqrt((1.0 - g * g) * params->rho * params->kT / kCs2); };
  s->sigma_s = sig(s->gamma_s);
  s->sigma_b = sig(s->gamma_b);
  s->sigma_g = sig(s->gamma_g);

  const size_t N = static_cast<size_t>(s->N);
  const size_t sz = s->ssize;
  bool ok = true;
  auto A = [&](size_t bytes) {
    void* ptr = dev_alloc(s, bytes);
    ok = ok && ptr;
    return ptr;
  };
  s->f[0] = A(sz * N * s->q);
  s->f[1] = A(sz * N * s->q);
  s->psi[0] = A(sz * N);
  s->psi[1] = A(sz * N);
  s->phi[0] = A(sz * N);
  s->phi[1] = A(sz * N);
  s->acc = A(sz * N);
  s->mu = A(sz * N);
  s->u = A(sz * N * s->d);
  s->noise = A(sz * N);
  // z-chunk of the tiled SMOL kernels: at least ~2048 blocks when possible.
  {
    const int bxy = ((params->nx + kTX - 1) / kTX) * ((params->ny + kTY - 1) / kTY);
    int zc = params->nz;
    while (zc > 8 && bxy * ((params->nz + zc - 1) / zc) < 2048) zc = (zc + 1) / 2;
    s->zc = std::max(1, zc);
  }
  s->nparts = std::min(1024, std::max(1, grid_for(s->N)));
  s->part = static_cast<double*>(A(sizeof(double) * 10 * s->nparts));
  s->tot = static_cast<double*>(A(sizeof(double) * 16));
  if (!ok) {
    std::string msg = "device allocation failed";
    release_all(s);
    delete s;
    return fail(nullptr, LBL_E_NOMEM, msg);
  }
  rc = hip_check(s, hipMemsetAsync(s->noise, 0, sz * N, s->stream), "clear noise");
  if (!rc) rc = select(s->p).init(s, init);
  if (!rc) rc = hip_check(s, hipStreamSynchronize(s->stream), "create sync");
  if (rc) {
    std::string msg = s->err;
    release_all(s);
    delete s;
    return fail(nullptr, rc, msg);
  }
  *out = s;
  return LBL_OK;
}

}  // namespace

extern "C" {

int lbl_abi_version(void) { return LBL_ABI_VERSION; }

const char* lbl_strerror(int status) {
  switch (status) {
    case LBL_OK: return "ok";
    case LBL_E_INVAL: return "invalid argument";
    case LBL_E_NOMEM: return "out of device memory";
    case LBL_E_DEVICE: return "HIP runtime error";
    case LBL_E_NONFINITE: return "non-finite conserved total";
    case LBL_E_BUFSIZE: return "destination buffer too small";
    case LBL_E_UNSUPPORTED: return "observable not available";
    default: return "unknown status";
  }
}

const char* lbl_last_error(const lbl_sim* sim) {
  return sim ? sim->err.c_str() : g_create_error.c_str();
}

int lbl_create(const lbl_params* params, const lbl_init* init, const lbl_env* env,
               lbl_sim** out) {
  try {
    g_create_error.clear();
    return create_impl(params, init, env, out);
  } catch (const std::exception& e) {
    return fail(nullptr, LBL_E_NOMEM, e.what());
  } catch (...) {
    return fail(nullptr, LBL_E_DEVICE, "unexpected exception");
  }
}

int lbl_step(lbl_sim* sim, int64_t nsteps) {
  if (!sim) return LBL_E_INVAL;
  if (nsteps < 0) return fail(sim, LBL_E_INVAL, "nsteps must be >= 0");
  try {
    if (int rc = hip_check(sim, hipSetDevice(sim->device), "hipSetDevice")) return rc;
    return select(sim->p).step(sim, nsteps);
  } catch (...) {
    return fail(sim, LBL_E_DEVICE, "unexpected exception in lbl_step");
  }
}

size_t lbl_observable_bytes(const lbl_sim* sim, int what) { return sim ? obs_bytes(sim, what) : 0; }

int lbl_observe(lbl_sim* sim, int what, void* dst, size_t bytes, int dst_is_device) {
  if (!sim) return LBL_E_INVAL;
  if (!dst) return fail(sim, LBL_E_INVAL, "dst must not be NULL");
  const size_t need = obs_bytes(sim, what);
  if (need == 0) return fail(sim, LBL_E_INVAL, "unknown observable");
  if (bytes < need) return fail(sim, LBL_E_BUFSIZE, "destination buffer too small");
  try {
    if (int rc = hip_check(sim, hipSetDevice(sim->device), "hipSetDevice")) return rc;
    if (sim->deferred) {
      const int rc = sim->deferred;
      sim->deferred = LBL_OK;
      return rc;
    }
    if (what == LBL_OBS_STEP || what == LBL_OBS_NSAMPLES) {
      int rc = hip_check(sim, hipStreamSynchronize(sim->stream), "observe sync");
      if (rc) return rc;
      const int64_t v = what == LBL_OBS_STEP ? sim->step : sim->nsamples;
      if (dst_is_device)
        return hip_check(sim, hipMemcpy(dst, &v, 8, hipMemcpyHostToDevice), "copy");
      std::memcpy(dst, &v, 8);
      return LBL_OK;
    }
    double* target = static_cast<double*>(dst);
    double* tmp = nullptr;
    if (!dst_is_device) {
      tmp = static_cast<double*>(dev_alloc(sim, need));
      if (!tmp) return fail(sim, LBL_E_NOMEM, "device allocation failed (observe staging)");
      target = tmp;
    }
    int rc = select(sim->p).observe(sim, what, target);
    if (rc == LBL_E_UNSUPPORTED) fail(sim, rc, "observable not available for this simulation");
    if (!rc && tmp)
      rc = hip_check(sim, hipMemcpyAsync(dst, tmp, need, hipMemcpyDeviceToHost, sim->stream),
                     "copy to host");
    if (!rc) rc = hip_check(sim, hipStreamSynchronize(sim->stream), "observe sync");
    dev_release(sim, tmp);
    if (!rc && what == LBL_OBS_TOTALS) {
      const double* t = static_cast<const double*>(dst);
      if (!dst_is_device) {
        for (int k = 0; k < 10; ++k)
          if (!std::isfinite(t[k])) return fail(sim, LBL_E_NONFINITE, "non-finite totals");
      }
    }
    return rc;
  } catch (...) {
    return fail(sim, LBL_E_DEVICE, "unexpected exception in lbl_observe");
  }
}

int lbl_timing_enable(lbl_sim* sim, int enable) {
  if (!sim) return LBL_E_INVAL;
  if (int rc = hip_check(sim, hipSetDevice(sim->device), "hipSetDevice")) return rc;
  if (int rc = drain_timing(sim)) return rc;
  for (auto& t : sim->kt) {
    t.launches = 0;
    t.total_ms = 0.0;
  }
  sim->kt.clear();
  sim->timing = enable != 0;
  return LBL_OK;
}

int lbl_timing_read(lbl_sim* sim, lbl_kernel_time* out, int max_entries, int* n_entries) {
  if (!sim || !n_entries || (max_entries > 0 && !out)) return LBL_E_INVAL;
  if (int rc = hip_check(sim, hipSetDevice(sim->device), "hipSetDevice")) return rc;
  if (int rc = drain_timing(sim)) return rc;
  const int n = static_cast<int>(sim->kt.size());
  for (int k = 0; k < n && k < max_entries; ++k) out[k] = sim->kt[k];
  *n_entries = n;
  return LBL_OK;
}

int lbl_destroy(lbl_sim* sim) {
  if (!sim) return LBL_OK;
  if (sim->stream || !sim->owned.empty()) (void)hipSetDevice(sim->device);
  (void)hipStreamSynchronize(sim->stream);
  destroy_events(sim);
  release_all(sim);
  delete sim;
  return LBL_OK;
}

}  // extern "C"
