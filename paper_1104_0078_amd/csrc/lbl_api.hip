// lbl_api.hip -- the C ABI of include/lbl.h: simulation lifecycle, parameter
// validation, device memory through the injected allocator, the per-step
// launch sequence of the coupled FLBE + SMOL sweep, observables, launch
// schedules, and the pool that batches independent simulations.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <mutex>
#include <array>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "lbl.h"
#include "lbl_kernels.hpp"
#include "lbl_observe.hpp"
#include "lbl_batch.hpp"

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
  void* u_end = nullptr;  // velocity of the streamed populations (stages at t_{n+1})
  void* noise = nullptr;
  void* fspec = nullptr;  // FD noise in Fourier space: half spectrum (interleaved re, im)
  void* famp = nullptr;   // and its amplitude table sqrt(-2 kT M L(q)) / N
  hipfftHandle fft_fwd = nullptr, fft_inv = nullptr;
  hipfftHandle fft_obs = nullptr;  // sample_full_k: psi -> half spectrum
  void* fk_spec = nullptr;         // its output (interleaved re, im)
  double* fk_acc = nullptr;        // sum over samples of |psi_q|^2 / N
  void* sig = nullptr;      // force_form STRESS: order-parameter stress, d(d+1)/2 components
  void* fstress = nullptr;  // and its divergence, the force density (d*N)
  double* part = nullptr;
  int nparts = 0;
  double* tot = nullptr;
  bool tot_pending = false;
  double* planes = nullptr;  // [kMaxFields][3][Lmax] plane sums
  double* col = nullptr;     // [kMaxFields][nz][nx] column sums
  double* sk = nullptr;      // [2][d][Lmax] sums of |psi_k|^2/N and of its square
  double* uk = nullptr;      // [2][d][d][Lmax] the same for each velocity component
  int64_t step = 0;
  int64_t nsamples = 0;
  uint32_t k0 = 0, k1 = 0;
  int zc = 1;       // planes per block of the z-marching SMOL stage kernels
  int zc_prep = 1;  // planes per block of the z-marching preparation kernel
  int zc_stress = 1;  // planes per block of the z-marching FV stress kernels (3-D)
  int zc_uend = 1;    // planes per block of the velocity pass with the noise (3-D)
  int lb_lw = 6;       // log2 of the LB block width along x
  int lb_swizzle = 0;  // XCD-contiguous block order: bit 0 LB kernels, bit 1 tile kernels
  int overlap = 0;     // 1: first RK stage on `aux`, concurrent with the velocity pass;
                       // 2: SMOL noise on `aux`, concurrent with the LB passes;
                       // 3: SMOL noise drawn inside the velocity pass (the default)
  hipStream_t aux = nullptr;  // created on first use (default priority)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
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
  if (s->fft_fwd) (void)hipfftDestroy(s->fft_fwd);
  if (s->fft_inv) (void)hipfftDestroy(s->fft_inv);
  if (s->fft_obs) (void)hipfftDestroy(s->fft_obs);
  s->fft_fwd = s->fft_inv = s->fft_obs = nullptr;
  for (void* ptr : s->owned) dev_free(s, ptr);
  s->owned.clear();
}

inline int grid_for(int n) { return (n + kBlock - 1) / kBlock; }
inline int grid_for64(int64_t n) { return static_cast<int>((n + kBlock - 1) / kBlock); }

// Values of the real-to-complex half spectrum: nz x ny x (nx/2 + 1).
size_t half_spectrum(const lbl_params& p) {
  return static_cast<size_t>(p.nx / 2 + 1) * p.ny * p.nz;
}


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

// Launch through `fn` on `stream`, bracketed by timing events when timing is
// on, and check the launch.
template <class Fn>
int launch_on(lbl_sim* s, hipStream_t stream, const char* name, Fn&& fn) {
  hipEvent_t a = nullptr, b = nullptr;
  if (s->timing) {
    a = take_event(s);
    b = take_event(s);
    if (a) (void)hipEventRecord(a, stream);
  }
  fn();
  const hipError_t e = hipGetLastError();
  if (s->timing && a && b) {
    (void)hipEventRecord(b, stream);
    s->pending.push_back(lbl_sim::Pending{kernel_slot(s, name), a, b});
  }
  return hip_check(s, e, name);
}

template <class Fn>
int launch(lbl_sim* s, const char* name, Fn&& fn) {
  return launch_on(s, s->stream, name, static_cast<Fn&&>(fn));
}

// Second stream and fork/join events for the concurrent first stage.  Work
// on `aux` is always joined back into the simulation's stream, so a
// synchronisation of that stream covers it.
int ensure_aux(lbl_sim* s) {
  if (s->aux) return LBL_OK;
  if (int rc = hip_check(s, hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking), "aux stream"))
    return rc;
  if (int rc = hip_check(s, hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming), "event"))
    return rc;
  return hip_check(s, hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming), "event");
}

void destroy_aux(lbl_sim* s) {
  if (s->aux) {
    (void)hipStreamSynchronize(s->aux);
    (void)hipStreamDestroy(s->aux);
  }
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->ev_join) (void)hipEventDestroy(s->ev_join);
  s->aux = nullptr;
  s->ev_fork = s->ev_join = nullptr;
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
  if (p->lattice != LBL_D2Q9 && p->lattice != LBL_D3Q15 && p->lattice != LBL_D3Q19)
    return fail(nullptr, LBL_E_INVAL, "lattice must be LBL_D2Q9, LBL_D3Q15 or LBL_D3Q19");
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
  if (p->lattice != LBL_D2Q9 && p->nz < 4) return fail(nullptr, LBL_E_INVAL, "nz must be >= 4");
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
  if (p->sample_every < 0) return fail(nullptr, LBL_E_INVAL, "sample_every must be >= 0");
  if (p->fd_noise != LBL_FDNOISE_LINK && p->fd_noise != LBL_FDNOISE_FOURIER)
    return fail(nullptr, LBL_E_INVAL, "fd_noise must be LBL_FDNOISE_LINK or LBL_FDNOISE_FOURIER");
  if (p->fd_noise == LBL_FDNOISE_FOURIER && p->smol != LBL_SMOL_FD)
    return fail(nullptr, LBL_E_INVAL, "Fourier-space noise is an option of the FD variant");
  if (p->force_form != LBL_FORCE_PSI_GRAD_MU && p->force_form != LBL_FORCE_STRESS)
    return fail(nullptr, LBL_E_INVAL,
                "force_form must be LBL_FORCE_PSI_GRAD_MU or LBL_FORCE_STRESS");
  if (p->sample_full_k != 0 && p->sample_full_k != 1)
    return fail(nullptr, LBL_E_INVAL, "sample_full_k must be 0 or 1");
  if (p->walls != LBL_WALLS_PERIODIC && p->walls != LBL_WALLS_LAST)
    return fail(nullptr, LBL_E_INVAL, "walls must be LBL_WALLS_PERIODIC or LBL_WALLS_LAST");
  if (p->reserved != 0) return fail(nullptr, LBL_E_INVAL, "reserved must be 0");
  for (int w = 0; w < 2; ++w)
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(p->u_wall[w][k]))
        return fail(nullptr, LBL_E_INVAL, "wall velocities must be finite");
  if (p->walls == LBL_WALLS_LAST) {
    if (p->smol != LBL_SMOL_FV)
      return fail(nullptr, LBL_E_INVAL, "walls are an option of the FV variant");
    if (p->force_form != LBL_FORCE_PSI_GRAD_MU)
      return fail(nullptr, LBL_E_INVAL, "walls need force_form LBL_FORCE_PSI_GRAD_MU");
    const int last = p->lattice == LBL_D2Q9 ? 1 : 2;
    if (p->u_wall[0][last] != 0.0 || p->u_wall[1][last] != 0.0)
      return fail(nullptr, LBL_E_INVAL, "walls move tangentially (no component along the "
                                        "last axis)");
  } else if (p->u_wall[0][0] != 0.0 || p->u_wall[0][1] != 0.0 || p->u_wall[0][2] != 0.0 ||
             p->u_wall[1][0] != 0.0 || p->u_wall[1][1] != 0.0 || p->u_wall[1][2] != 0.0) {
    return fail(nullptr, LBL_E_INVAL, "wall velocities need walls");
  }
  if (in->kind < LBL_INIT_REST || in->kind > LBL_INIT_USER)
    return fail(nullptr, LBL_E_INVAL, "unknown init kind");
  if (in->kind == LBL_INIT_TANH_2IF && !(p->a < 0 && p->b > 0 && p->kappa > 0))
    return fail(nullptr, LBL_E_INVAL, "two-phase init needs a < 0 < b and kappa > 0");
  if (in->kind == LBL_INIT_USER && (!in->psi0 || !in->f0))
    return fail(nullptr, LBL_E_INVAL, "USER init needs psi0 and f0");
  if (!std::isfinite(in->psi_std) || in->psi_std < 0)
    return fail(nullptr, LBL_E_INVAL, "psi_std must be finite and >= 0");
  if (in->step0 < 0 || in->step0 > 0xffffffffLL)
    return fail(nullptr, LBL_E_INVAL, "step0 must lie in [0, 2^32)");
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

  // Default z-chunks of the tiled SMOL kernels (3-D): as many chunks as fill
  // the device's resident block slots of each kernel in whole rounds, one
  // round for the stage kernel, two for the preparation kernel and the
  // velocity pass with the noise (measured best on 256^3), and never fewer
  // than 8 planes per chunk.
  static int default_chunks(lbl_sim* s) {
    if (Lat<Q>::D != 3) return LBL_OK;
    int cus = 0, nb_stage = 0, nb_prep = 0;
    int rc = hip_check(s, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                                s->device), "CU count");
    if (!rc) {
      if (SMOL == kFV) {
        rc = hip_check(s, hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb_stage, k_stage_fv<S, Q>,
                                                                       kTX * kTY, 0), "occupancy");
        if (!rc)
          rc = hip_check(s, hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb_prep, k_prep_fv<S, Q>,
                                                                         kTX * kTY, 0), "occupancy");
      } else {
        rc = hip_check(s, hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb_stage, k_stage_fd<S, Q>,
                                                                       kTX * kTY, 0), "occupancy");
        if (!rc)
          rc = hip_check(s, hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb_prep, k_prep_fd<S, Q>,
                                                                         kTX * kTY, 0), "occupancy");
      }
    }
    int nb_stress = 0, nb_uend = 0;
    if constexpr (SMOL == kFV && Lat<Q>::D == 3)
      if (!rc)
        rc = hip_check(s, hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &nb_stress, k_stress_force_fv3<S, Q>, kTX * kTY, 0),
                       "occupancy");
    if (!rc)
      rc = hip_check(s, hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &nb_uend, k_uend_noise<S, DEV, Q, SMOL, false>, kTX * kTY, 0),
                     "occupancy");
    if (rc) return rc;
    const int nz = s->p.nz;
    const long bxy = static_cast<long>((s->p.nx + kTX - 1) / kTX) * ((s->p.ny + kTY - 1) / kTY);
    auto pick = [&](int per_cu, int rounds) {
      const long slots = static_cast<long>(std::max(1, per_cu)) * std::max(1, cus) * rounds;
      const long chunks = std::max(1L, (slots + bxy - 1) / bxy);
      const int zc = static_cast<int>((nz + chunks - 1) / chunks);
      return std::min(nz, std::max(8, zc));
    };
    s->zc = pick(nb_stage, 1);
    s->zc_prep = pick(nb_prep, 2);
    s->zc_stress = pick(nb_stress, 2);
    s->zc_uend = pick(nb_uend, 2);
    return LBL_OK;
  }

  static bool fourier(const lbl_sim* s) {
    return SMOL == kFD && s->p.fd_noise == LBL_FDNOISE_FOURIER;
  }

  static int fft_check(lbl_sim* s, hipfftResult r, const char* what) {
    if (r == HIPFFT_SUCCESS) return LBL_OK;
    return fail(s, LBL_E_DEVICE, std::string(what) + ": hipFFT error " + std::to_string(r));
  }

  // FD noise in Fourier space: plans of the real-to-complex pair on the
  // simulation's stream and the amplitude table, once per simulation.
  static int fourier_setup(lbl_sim* s) {
    if (!fourier(s)) return LBL_OK;
    constexpr bool dbl = sizeof(S) == 8;
    const hipfftType tf = dbl ? HIPFFT_D2Z : HIPFFT_R2C, ti = dbl ? HIPFFT_Z2D : HIPFFT_C2R;
    const lbl_params& p = s->p;
    for (int k = 0; k < 2; ++k) {
      hipfftHandle& h = k == 0 ? s->fft_fwd : s->fft_inv;
      const hipfftType t = k == 0 ? tf : ti;
      // x varies fastest: the transform's dimensions are (nz, ny, nx).
      const hipfftResult r = Lat<Q>::D == 3 ? hipfftPlan3d(&h, p.nz, p.ny, p.nx, t)
                                            : hipfftPlan2d(&h, p.ny, p.nx, t);
      if (r != HIPFFT_SUCCESS) h = nullptr;
      if (int rc = fft_check(s, r, "hipfftPlan")) return rc;
      if (int rc = fft_check(s, hipfftSetStream(h, s->stream), "hipfftSetStream")) return rc;
    }
    const int nh = static_cast<int>(half_spectrum(p));
    const Geom g = geom(s);
    const double two_kT_M = 2.0 * p.kT * p.M;
    S* amp = static_cast<S*>(s->famp);
    k_fourier_amp<S, Lat<Q>::D><<<(nh + 255) / 256, 256, 0, s->stream>>>(g, two_kT_M, amp);
    return launched(s, "k_fourier_amp");
  }

  // N^n = F^-1[ amp F[w] ] into s->noise.
  static int fourier_noise(lbl_sim* s, uint32_t step) {
    S* w = static_cast<S*>(s->noise);
    S* spec = static_cast<S*>(s->fspec);
    const int nh = static_cast<int>(half_spectrum(s->p));
    const hipStream_t st = s->stream;
    if (int rc = launch(s, "k_white", [&] {
          k_white<S><<<(s->N + 255) / 256, 256, 0, st>>>(s->N, step, s->k0, s->k1, w);
        }))
      return rc;
    hipfftResult r = HIPFFT_SUCCESS;
    if (int rc = launch(s, "fft", [&] {
          if constexpr (sizeof(S) == 8)
            r = hipfftExecD2Z(s->fft_fwd, reinterpret_cast<hipfftDoubleReal*>(w),
                              reinterpret_cast<hipfftDoubleComplex*>(spec));
          else
            r = hipfftExecR2C(s->fft_fwd, reinterpret_cast<hipfftReal*>(w),
                              reinterpret_cast<hipfftComplex*>(spec));
        }))
      return rc;
    if (int rc = fft_check(s, r, "forward FFT")) return rc;
    if (int rc = launch(s, "k_fourier_scale", [&] {
          k_fourier_scale<S><<<(nh + 255) / 256, 256, 0, st>>>(
              nh, static_cast<const S*>(s->famp), spec);
        }))
      return rc;
    if (int rc = launch(s, "fft", [&] {
          if constexpr (sizeof(S) == 8)
            r = hipfftExecZ2D(s->fft_inv, reinterpret_cast<hipfftDoubleComplex*>(spec),
                              reinterpret_cast<hipfftDoubleReal*>(w));
          else
            r = hipfftExecC2R(s->fft_inv, reinterpret_cast<hipfftComplex*>(spec),
                              reinterpret_cast<hipfftReal*>(w));
        }))
      return rc;
    return fft_check(s, r, "inverse FFT");
  }

  // Whole-zone spectrum of psi at every sample (sample_full_k): a
  // real-to-complex plan of psi's storage type and a cleared FP64 accumulator.
  static int full_k_setup(lbl_sim* s) {
    if (!s->p.sample_full_k) return LBL_OK;
    constexpr hipfftType t = sizeof(S) == 8 ? HIPFFT_D2Z : HIPFFT_R2C;
    const lbl_params& p = s->p;
    const hipfftResult r = Lat<Q>::D == 3 ? hipfftPlan3d(&s->fft_obs, p.nz, p.ny, p.nx, t)
                                          : hipfftPlan2d(&s->fft_obs, p.ny, p.nx, t);
    if (r != HIPFFT_SUCCESS) s->fft_obs = nullptr;
    if (int rc = fft_check(s, r, "hipfftPlan")) return rc;
    if (int rc = fft_check(s, hipfftSetStream(s->fft_obs, s->stream), "hipfftSetStream"))
      return rc;
    return hip_check(s, hipMemsetAsync(s->fk_acc, 0, sizeof(double) * half_spectrum(p), s->stream),
                     "clear full-k accumulator");
  }

  // Add |psi_q|^2 / N of the current psi to the whole-zone accumulator.  psi
  // is copied into a Runge-Kutta stage buffer first (dead between steps), so
  // that the transform cannot touch the state.
  static int full_k_sample(lbl_sim* s) {
    const size_t bytes = sizeof(S) * static_cast<size_t>(s->N);
    S* work = static_cast<S*>(s->phi[0]);
    if (int rc = hip_check(s, hipMemcpyAsync(work, s->psi[s->pcur], bytes, hipMemcpyDeviceToDevice,
                                             s->stream), "copy psi"))
      return rc;
    hipfftResult r = HIPFFT_SUCCESS;
    if (int rc = launch(s, "fft", [&] {
          if constexpr (sizeof(S) == 8)
            r = hipfftExecD2Z(s->fft_obs, reinterpret_cast<hipfftDoubleReal*>(work),
                              reinterpret_cast<hipfftDoubleComplex*>(s->fk_spec));
          else
            r = hipfftExecR2C(s->fft_obs, reinterpret_cast<hipfftReal*>(work),
                              reinterpret_cast<hipfftComplex*>(s->fk_spec));
        }))
      return rc;
    if (int rc = fft_check(s, r, "full-k FFT")) return rc;
    const int nh = static_cast<int>(half_spectrum(s->p));
    const double scale = 1.0 / static_cast<double>(s->N);
    return launch(s, "k_sample", [&] {
      k_power_acc<S><<<(nh + 255) / 256, 256, 0, s->stream>>>(
          nh, static_cast<const S*>(s->fk_spec), scale, s->fk_acc);
    });
  }

  static int init(lbl_sim* s, const lbl_init* in) {
    if (int rc = default_chunks(s)) return rc;
    if (int rc = fourier_setup(s)) return rc;
    if (int rc = full_k_setup(s)) return rc;
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
      k_scatter_user<S, DEV, Q><<<grid, kBlock, 0, s->stream>>>(g, wall_spec(s), f0, f);
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
        g, wall_spec(s), in->boost_u[0], in->boost_u[1], Lat<Q>::D == 3 ? in->boost_u[2] : 0.0, f);
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
    a.Fext = force && s->p.force_form == LBL_FORCE_STRESS ? static_cast<const S*>(s->fstress)
                                                          : nullptr;
    a.noise = s->p.kT > 0;
    a.nt = 2.0 * sizeof(S) * s->q * static_cast<double>(s->N) > kStreamBytes;
    for (int w = 0; w < 2; ++w)
      for (int k = 0; k < 3; ++k) a.uw[w][k] = S(s->p.u_wall[w][k]);
    return a;
  }

  static WallSpec wall_spec(const lbl_sim* s) {
    WallSpec w;
    w.on = s->p.walls == LBL_WALLS_LAST;
    w.rho0 = s->p.rho;
    for (int k = 0; k < 2; ++k)
      for (int c = 0; c < 3; ++c) w.u[k][c] = s->p.u_wall[k][c];
    return w;
  }

  static dim3 site_grid(const lbl_sim* s) {
    return dim3((s->p.nx + kBX - 1) / kBX, (s->p.ny + kBY - 1) / kBY, s->p.nz);
  }

  static int launch_lb(lbl_sim* s, const LBArgs<S>& a, bool collide, const char* name) {
    const SiteMap m = make_site_map(s->p.nx, s->p.ny, s->p.nz, s->lb_lw, (s->lb_swizzle & 1) != 0);
    const dim3 grid(site_map_blocks(m)), block(kSiteBlock);
    const bool ghost = s->gamma_g != 0.0;
    const hipStream_t st = s->stream;
    if (s->p.walls == LBL_WALLS_LAST) {
      return launch(s, name, [&] {
        if (!collide) {
          if (a.nt)
            k_lb<S, DEV, Q, SMOL, false, false, true, true><<<grid, block, 0, st>>>(a, m);
          else
            k_lb<S, DEV, Q, SMOL, false, false, false, true><<<grid, block, 0, st>>>(a, m);
        } else if (ghost) {
          k_lb<S, DEV, Q, SMOL, true, true, false, true><<<grid, block, 0, st>>>(a, m);
        } else if (a.nt) {
          k_lb<S, DEV, Q, SMOL, false, true, true, true><<<grid, block, 0, st>>>(a, m);
        } else {
          k_lb<S, DEV, Q, SMOL, false, true, false, true><<<grid, block, 0, st>>>(a, m);
        }
      });
    }
    return launch(s, name, [&] {
      if (!collide) {
        if (a.nt)
          k_lb<S, DEV, Q, SMOL, false, false, true><<<grid, block, 0, st>>>(a, m);
        else
          k_lb<S, DEV, Q, SMOL, false, false, false><<<grid, block, 0, st>>>(a, m);
      } else if (ghost) {
        if (a.nt)
          k_lb<S, DEV, Q, SMOL, true, true, true><<<grid, block, 0, st>>>(a, m);
        else
          k_lb<S, DEV, Q, SMOL, true, true, false><<<grid, block, 0, st>>>(a, m);
      } else {
        if (a.nt)
          k_lb<S, DEV, Q, SMOL, false, true, true><<<grid, block, 0, st>>>(a, m);
        else
          k_lb<S, DEV, Q, SMOL, false, true, false><<<grid, block, 0, st>>>(a, m);
      }
    });
  }

  // Force density as the divergence of the order-parameter stress of psi
  // into s->fstress (force_form STRESS).
  static int stress_force(lbl_sim* s, const S* psi) {
    const dim3 grid = site_grid(s), block(kBX, kBY);
    const Geom g = geom(s);
    const Coef<S> c = coef(s);
    S* sig = static_cast<S*>(s->sig);
    S* F = static_cast<S*>(s->fstress);
    if constexpr (SMOL == kFV && Lat<Q>::D == 3) {
      // one z-marching pass (the FV gradient spans 18 neighbours); sigma
      // stays on the chip
      const TileMap tm = make_tile_map(s->p.nx, s->p.ny, (s->p.nz + s->zc_stress - 1) / s->zc_stress,
                                       (s->lb_swizzle & 2) != 0);
      const dim3 tg(tile_map_blocks(tm)), tb(kTX, kTY);
      const int zc = s->zc_stress;
      return launch(s, "k_stress_force", [&] {
        k_stress_force_fv3<S, Q><<<tg, tb, 0, s->stream>>>(g, c, psi, F, zc, tm);
      });
    }
    if (int rc = launch(s, "k_stress", [&] {
          k_stress<S, Q, SMOL><<<grid, block, 0, s->stream>>>(g, c, psi, sig);
        }))
      return rc;
    return launch(s, "k_force_stress", [&] {
      k_force_stress<S, Q, SMOL><<<grid, block, 0, s->stream>>>(g, sig, F);
    });
  }

  // The FV stage kernel, in the fixed form `form` on 3-D lattices.
  template <bool WALLS>
  static int launch_stage_fv(lbl_sim* s, hipStream_t ss, const StageArgs<S>& a,
                             const TileMap& tm, dim3 tg, dim3 tb, int form) {
    if constexpr (Lat<Q>::D == 3) {
      if (form == kStageHeun1)
        return launch_on(s, ss, "k_stage", [&] {
          k_stage_fv<S, Q, WALLS, kStageHeun1><<<tg, tb, 0, ss>>>(a, tm);
        });
      if (form == kStageHeun2)
        return launch_on(s, ss, "k_stage", [&] {
          k_stage_fv<S, Q, WALLS, kStageHeun2><<<tg, tb, 0, ss>>>(a, tm);
        });
    }
    return launch_on(s, ss, "k_stage", [&] { k_stage_fv<S, Q, WALLS><<<tg, tb, 0, ss>>>(a, tm); });
  }

  // The velocity pass with the SMOL noise N^n of step `la.step`, on the
  // SMOL tiles (z-chunks of zc_uend planes in 3-D).
  static int launch_uend_noise(lbl_sim* s, const LBArgs<S>& la, S* noise) {
    constexpr bool k3 = Lat<Q>::D == 3;
    PrepArgs<S> pa;
    pa.g = la.g;
    pa.c = coef(s);
    pa.amp = S(std::sqrt(2.0 * s->p.kT * s->p.M));
    pa.k0 = s->k0;
    pa.k1 = s->k1;
    pa.step = la.step;
    pa.zc = k3 ? s->zc_uend : 1;
    pa.psi = nullptr;
    pa.noise = noise;
    pa.mu = nullptr;
    const TileMap tm = make_tile_map(s->p.nx, s->p.ny,
                                     k3 ? (s->p.nz + s->zc_uend - 1) / s->zc_uend : 1,
                                     (s->lb_swizzle & 2) != 0);
    const dim3 tg(tile_map_blocks(tm)), tb(kTX, kTY);
    const hipStream_t st = s->stream;
    if constexpr (SMOL == kFV) {
      if (s->p.walls == LBL_WALLS_LAST)
        return launch(s, "k_uend", [&] {
          if (la.nt)
            k_uend_noise<S, DEV, Q, SMOL, true, true><<<tg, tb, 0, st>>>(la, pa, tm);
          else
            k_uend_noise<S, DEV, Q, SMOL, false, true><<<tg, tb, 0, st>>>(la, pa, tm);
        });
    }
    return launch(s, "k_uend", [&] {
      if (la.nt)
        k_uend_noise<S, DEV, Q, SMOL, true><<<tg, tb, 0, st>>>(la, pa, tm);
      else
        k_uend_noise<S, DEV, Q, SMOL, false><<<tg, tb, 0, st>>>(la, pa, tm);
    });
  }

  static int launch_mu(lbl_sim* s, const S* phi, S* mu) {
    const dim3 grid = site_grid(s), block(kBX, kBY);
    const Geom g = geom(s);
    const Coef<S> c = coef(s);
    if (s->p.walls == LBL_WALLS_LAST)
      return launch(s, "k_mu_w",
                    [&] { k_mu_w<S, Q><<<grid, block, 0, s->stream>>>(g, c, phi, mu); });
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
    const TileMap tm = make_tile_map(s->p.nx, s->p.ny,
                                     Lat<Q>::D == 3 ? (s->p.nz + s->zc - 1) / s->zc : 1,
                                     (s->lb_swizzle & 2) != 0);
    const TileMap tmp = make_tile_map(s->p.nx, s->p.ny,
                                      Lat<Q>::D == 3 ? (s->p.nz + s->zc_prep - 1) / s->zc_prep : 1,
                                      (s->lb_swizzle & 2) != 0);
    const dim3 tg(tile_map_blocks(tm)), tgp(tile_map_blocks(tmp)), tb(kTX, kTY);
    const bool want_noise = cpl != LBL_LB_ONLY && s->p.kT > 0;
    const bool prep_noise = want_noise && !fourier(s);
    const bool stress = cpl == LBL_FULL && s->p.force_form == LBL_FORCE_STRESS;
    const bool want_mu = cpl == LBL_FULL && !stress;
    if (stress)
      if (int rc = stress_force(s, psin)) return rc;
    if (want_noise && !prep_noise)
      if (int rc = fourier_noise(s, n)) return rc;
    // With overlap 2 the SMOL noise (arithmetic-bound: the Box-Muller
    // normals) is drawn on the second stream while the memory-bound LB
    // passes run here; it depends on the counter only, and the previous
    // step's stages, its last readers, precede the fork.  Joined before the
    // first stage.
    const bool walls = s->p.walls == LBL_WALLS_LAST;
    // Walls (an FV option) run the tiled SMOL kernels with the wall rules.
    constexpr bool kTiledWalls = SMOL == kFV;
    const bool walls_tiled = walls && kTiledWalls;
    const bool split = prep_noise && s->overlap == 2;
    // The velocity of the streamed populations is needed by the stages at
    // t_{n+1}; with overlap 3 the same pass draws the SMOL noise, which the
    // first stage is the first to read.
    const bool uend = cpl == LBL_FULL && s->p.rk_stages > 1;
    const bool fuse = prep_noise && uend && s->overlap == 3;
    if (split) {
      if (int rc = ensure_aux(s)) return rc;
      if (int rc = hip_check(s, hipEventRecord(s->ev_fork, s->stream), "fork")) return rc;
      if (int rc = hip_check(s, hipStreamWaitEvent(s->aux, s->ev_fork, 0), "fork")) return rc;
    }
    for (int part = split ? 0 : 1; part < 2; ++part) {
      // part 0: the noise alone on `aux`; part 1: what remains on the stream
      const bool do_noise = prep_noise && !fuse && (part == 0 || !split);
      const bool do_mu = want_mu && part == 1;
      if (!do_noise && !do_mu) continue;
      const hipStream_t ps = part == 0 ? s->aux : s->stream;
      PrepArgs<S> pa;
      pa.g = g;
      pa.c = coef(s);
      pa.amp = S(std::sqrt(2.0 * s->p.kT * s->p.M));
      pa.k0 = s->k0;
      pa.k1 = s->k1;
      pa.step = n;
      pa.zc = s->zc_prep;
      pa.psi = psin;
      pa.noise = do_noise ? noise : nullptr;
      pa.mu = do_mu ? static_cast<S*>(s->mu) : nullptr;
      const char* name = part == 0 ? "k_prep_noise" : "k_prep";
      int rc;
      if constexpr (kTiledWalls) {
        if (walls_tiled)
          rc = launch_on(s, ps, name,
                         [&] { k_prep_fv<S, Q, true><<<tgp, tb, 0, ps>>>(pa, tmp); });
        else
          rc = launch_on(s, ps, name, [&] { k_prep_fv<S, Q><<<tgp, tb, 0, ps>>>(pa, tmp); });
      } else if (SMOL == kFV)
        rc = launch_on(s, ps, name, [&] { k_prep_fv<S, Q><<<tgp, tb, 0, ps>>>(pa, tmp); });
      else
        rc = launch_on(s, ps, name, [&] { k_prep_fd<S, Q><<<tgp, tb, 0, ps>>>(pa, tmp); });
      if (rc) return rc;
      if (part == 0)
        if (int rc2 = hip_check(s, hipEventRecord(s->ev_join, s->aux), "join")) return rc2;
    }
    if (cpl != LBL_SMOL_ONLY) {
      const LBArgs<S> a = lb_args(s, fin, fout, psin, u, cpl == LBL_FULL, n);
      if (int rc = launch_lb(s, a, true, "k_lb")) return rc;
    }
    // The velocity of the streamed populations (for the stages at t_{n+1})
    // and the first stage (at t_n) are independent: with `overlap` 1 the first
    // stage runs on the second stream while the velocity pass runs here.
    const bool fork = uend && s->overlap == 1;
    if (fork) {
      if (int rc = ensure_aux(s)) return rc;
      if (int rc = hip_check(s, hipEventRecord(s->ev_fork, s->stream), "fork")) return rc;
      if (int rc = hip_check(s, hipStreamWaitEvent(s->aux, s->ev_fork, 0), "fork")) return rc;
    }
    if (uend && !fork) {
      const LBArgs<S> a = lb_args(s, fout, nullptr, psin, static_cast<S*>(s->u_end), 1, n);
      if (fuse) {
        if (int rc = launch_uend_noise(s, a, noise)) return rc;
      } else if (int rc = launch_lb(s, a, false, "k_uend")) {
        return rc;
      }
    }
    if (split)
      if (int rc = hip_check(s, hipStreamWaitEvent(s->stream, s->ev_join, 0), "join")) return rc;
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
        a.u_end = static_cast<const S*>(s->u_end);
        a.utime = st == 0 ? kAtN : (st == ns - 1 ? kAtN1 : kAtMid);
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
        const hipStream_t ss = (fork && st == 0) ? s->aux : s->stream;
        int rc;
        // Heun under full coupling: its two stages as fixed forms (3-D FV)
        int form = kStageAny;
        if (ns == 2 && cpl == LBL_FULL) form = st == 0 ? kStageHeun1 : kStageHeun2;
        if constexpr (kTiledWalls) {
          if (walls_tiled)
            rc = launch_stage_fv<true>(s, ss, a, tm, tg, tb, form);
          else
            rc = launch_stage_fv<false>(s, ss, a, tm, tg, tb, form);
        } else if (SMOL == kFV)
          rc = launch_on(s, ss, "k_stage", [&] { k_stage_fv<S, Q><<<tg, tb, 0, ss>>>(a, tm); });
        else
          rc = launch_on(s, ss, "k_stage", [&] { k_stage_fd<S, Q><<<tg, tb, 0, ss>>>(a, tm); });
        if (rc) return rc;
        if (fork && st == 0) {
          if (int rc2 = hip_check(s, hipEventRecord(s->ev_join, s->aux), "join")) return rc2;
          const LBArgs<S> b = lb_args(s, fout, nullptr, psin, static_cast<S*>(s->u_end), 1, n);
          if (int rc2 = launch_lb(s, b, false, "k_uend")) return rc2;
          if (int rc2 = hip_check(s, hipStreamWaitEvent(s->stream, s->ev_join, 0), "join"))
            return rc2;
        }
        phi = a.out;
      }
      s->pcur = 1 - s->pcur;
    }
    if (cpl != LBL_SMOL_ONLY) s->cur = 1 - s->cur;
    s->step += 1;
    if (s->p.sample_every > 0 && s->step % s->p.sample_every == 0) {
      if (int rc = sample(s, true, nullptr)) return rc;
      if (s->p.sample_full_k)
        if (int rc = full_k_sample(s)) return rc;
      if (int rc = totals(s, s->tot)) return rc;
      s->tot_pending = true;
      s->nsamples += 1;
    }
    return LBL_OK;
  }

  // Plane sums and axis DFTs of psi (and u when accumulating): adds
  // |X|^2/N into sk/uk when `accumulate`, writes psi's complex X into `cur`.
  static int sample(lbl_sim* s, bool accumulate, double* cur) {
    const Geom g = geom(s);
    const int D = Lat<Q>::D;
    FieldSet<S> fs{};
    fs.f[0] = static_cast<const S*>(s->psi[s->pcur]);
    fs.nf = 1;
    if (accumulate && s->p.coupling != LBL_SMOL_ONLY) {
      for (int b = 0; b < D; ++b) fs.f[1 + b] = static_cast<const S*>(s->u) + static_cast<size_t>(b) * s->N;
      fs.nf = 1 + D;
    }
    const int Lmax = s->Lmax;
    const int last = D - 1, Llast = D == 3 ? s->p.nz : s->p.ny;
    double* planes = s->planes;
    double* col = s->col;
    if (int rc = launch(s, "k_sample", [&] {
          k_plane_last<S><<<Llast, kRedBlock, 0, s->stream>>>(g, fs, last, Lmax, planes);
        }))
      return rc;
    if (D == 3)
      if (int rc = launch(s, "k_sample", [&] {
            k_plane_y<S><<<s->p.ny, kRedBlock, 0, s->stream>>>(g, fs, Lmax, planes);
          }))
        return rc;
    const dim3 gx1((s->p.nx + kRedBlock - 1) / kRedBlock, s->p.nz);
    if (int rc = launch(s, "k_sample",
                        [&] { k_plane_x1<S><<<gx1, kRedBlock, 0, s->stream>>>(g, fs, col); }))
      return rc;
    const int nf = fs.nf;
    if (int rc = launch(s, "k_sample", [&] {
          k_plane_x2<<<(s->p.nx + kRedBlock - 1) / kRedBlock, kRedBlock, 0, s->stream>>>(
              g, nf, col, Lmax, planes);
        }))
      return rc;
    const int nthreads = nf * D * Lmax;
    double* sk = accumulate ? s->sk : nullptr;
    double* uk = accumulate ? s->uk : nullptr;
    return launch(s, "k_sample", [&] {
      k_axis_dft<<<(nthreads + kRedBlock - 1) / kRedBlock, kRedBlock, 0, s->stream>>>(
          g, D, nf, Lmax, planes, sk, uk, cur);
    });
  }

  static int totals(lbl_sim* s, double* dst) {
    const Geom g = geom(s);
    const S* f = static_cast<const S*>(s->f[s->cur]);
    const S* psi = static_cast<const S*>(s->psi[s->pcur]);
    k_totals_partial<S, DEV, Q><<<s->nparts, kTotBlock, 0, s->stream>>>(g, wall_spec(s), f, psi,
                                                                       s->part);
    if (int rc = launched(s, "k_totals_partial")) return rc;
    k_totals_final<<<1, 64, 0, s->stream>>>(s->nparts, s->part, dst);
    return launched(s, "k_totals_final");
  }

  static int steps(lbl_sim* s, int64_t nsteps) {
    for (int64_t k = 0; k < nsteps; ++k)
      if (int rc = one_step(s)) return rc;
    return LBL_OK;
  }

  // Descriptor of a simulation for the batched kernels.
  static Replica<S> replica(const lbl_sim* s, int zc) {
    Replica<S> r;
    r.g = geom(s);
    r.c = coef(s);
    r.zc = zc;
    r.coupling = s->p.coupling;
    r.noise_on = s->p.kT > 0;
    for (int k = 0; k < 2; ++k) {
      r.f[k] = static_cast<S*>(s->f[k]);
      r.psi[k] = static_cast<S*>(s->psi[k]);
      r.phi[k] = static_cast<S*>(s->phi[k]);
    }
    r.acc = static_cast<S*>(s->acc);
    r.mu = static_cast<S*>(s->mu);
    r.u = static_cast<S*>(s->u);
    r.u_end = static_cast<S*>(s->u_end);
    r.noise = static_cast<S*>(s->noise);
    r.rho0 = S(s->p.rho);
    r.gamma_s = S(s->gamma_s);
    r.gamma_b = S(s->gamma_b);
    r.gamma_g = S(s->gamma_g);
    r.sigma_s = S(s->sigma_s);
    r.sigma_b = S(s->sigma_b);
    r.sigma_g = S(s->sigma_g);
    r.amp = S(std::sqrt(2.0 * s->p.kT * s->p.M));
    r.u0 = S(s->p.u_imposed[0]);
    r.u1 = S(s->p.u_imposed[1]);
    r.u2 = S(Lat<Q>::D == 3 ? s->p.u_imposed[2] : 0.0);
    for (int k = 0; k < 2; ++k)
      for (int c = 0; c < 3; ++c) r.uw[k][c] = S(s->p.u_wall[k][c]);
    r.k0 = s->k0;
    r.k1 = s->k1;
    return r;
  }

  static size_t replica_bytes() { return sizeof(Replica<S>); }

  // Fill the descriptor array for `sims` (host memory, replica_bytes() each)
  // and the two work tables.
  static void tables(const std::vector<lbl_sim*>& sims, int zc_override, int lb_lw,
                     void* reps_host, std::vector<Work>& wlb, std::vector<Work>& wtile) {
    const int lbw = 1 << lb_lw, lbh = kSiteBlock >> lb_lw;
    Replica<S>* reps = static_cast<Replica<S>*>(reps_host);
    wlb.clear();
    wtile.clear();
    for (size_t i = 0; i < sims.size(); ++i) {
      const lbl_sim* s = sims[i];
      const int zc = (Lat<Q>::D == 3 && zc_override > 0) ? std::min(zc_override, s->p.nz) : s->zc;
      reps[i] = replica(s, zc);
      const int rep = static_cast<int>(i);
      for (int bz = 0; bz < s->p.nz; ++bz)
        for (int by = 0; by < (s->p.ny + lbh - 1) / lbh; ++by)
          for (int bx = 0; bx < (s->p.nx + lbw - 1) / lbw; ++bx) wlb.push_back(Work{rep, bx, by, bz});
      const int nzc = Lat<Q>::D == 3 ? (s->p.nz + zc - 1) / zc : 1;
      for (int bz = 0; bz < nzc; ++bz)
        for (int by = 0; by < (s->p.ny + kTY - 1) / kTY; ++by)
          for (int bx = 0; bx < (s->p.nx + kTX - 1) / kTX; ++bx) wtile.push_back(Work{rep, bx, by, bz});
    }
  }

  // Enqueue `nsteps` batched steps of a group on `stream` (captured by the
  // caller into a graph).  The launches of step k take k; the replicas'
  // states move once, after the last step.
  static int enqueue_group(hipStream_t stream, const void* reps_dev, RepState* states, int nrep,
                           const Work* wlb, int nlb, int lb_lw, const Work* wtile, int ntile,
                           int rk, bool ghost, int nt, bool walls, int64_t nsteps) {
    if (nsteps < 0 || nsteps > (1 << 30)) return LBL_E_INVAL;
    if constexpr (SMOL == kFV)
      if (walls)
        return enqueue_steps<true>(stream, reps_dev, states, nrep, wlb, nlb, lb_lw, wtile, ntile,
                                   rk, ghost, nt, static_cast<int>(nsteps));
    if (walls) return LBL_E_INVAL;
    return enqueue_steps<false>(stream, reps_dev, states, nrep, wlb, nlb, lb_lw, wtile, ntile, rk,
                                ghost, nt, static_cast<int>(nsteps));
  }

  // WALLS: every replica of the group has walls (FV only; the ghost-rate
  // variant of the LB pass keeps the default cache policy there).
  template <bool WALLS>
  static int enqueue_steps(hipStream_t stream, const void* reps_dev, RepState* states, int nrep,
                           const Work* wlb, int nlb, int lb_lw, const Work* wtile, int ntile,
                           int rk, bool ghost, int nt, int nsteps) {
    const Replica<S>* reps = static_cast<const Replica<S>*>(reps_dev);
    const dim3 bsite(kSiteBlock), btile(kTX, kTY);
    for (int k = 0; k < nsteps; ++k) {
      kb_prep<S, Q, SMOL, WALLS><<<ntile, btile, 0, stream>>>(reps, states, wtile, k);
      bool ghost_nt = false;
      if constexpr (!WALLS) ghost_nt = ghost && nt;
      if (ghost_nt) {
        if constexpr (!WALLS)
          kb_lb<S, DEV, Q, SMOL, true, true><<<nlb, bsite, 0, stream>>>(reps, states, wlb, lb_lw,
                                                                          k);
      } else if (ghost)
        kb_lb<S, DEV, Q, SMOL, true, false, WALLS><<<nlb, bsite, 0, stream>>>(reps, states, wlb,
                                                                                lb_lw, k);
      else if (nt)
        kb_lb<S, DEV, Q, SMOL, false, true, WALLS><<<nlb, bsite, 0, stream>>>(reps, states, wlb,
                                                                                lb_lw, k);
      else
        kb_lb<S, DEV, Q, SMOL, false, false, WALLS><<<nlb, bsite, 0, stream>>>(reps, states, wlb,
                                                                                 lb_lw, k);
      // the velocity pass and the SMOL noise on the SMOL tiles
      if (nt)
        kb_uend_noise<S, DEV, Q, SMOL, true, WALLS><<<ntile, btile, 0, stream>>>(reps, states,
                                                                                  wtile, rk, k);
      else
        kb_uend_noise<S, DEV, Q, SMOL, false, WALLS><<<ntile, btile, 0, stream>>>(reps, states,
                                                                                   wtile, rk, k);
      for (int st = 0; st < rk; ++st)
        kb_stage<S, Q, SMOL, WALLS><<<ntile, btile, 0, stream>>>(reps, states, wtile, st, rk, k);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return LBL_E_DEVICE;
    }
    kb_advance<S><<<(nrep + 255) / 256, 256, 0, stream>>>(reps, states, nrep, nsteps);
    return hipGetLastError() == hipSuccess ? LBL_OK : LBL_E_DEVICE;
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
        k_gather<S, DEV, Q><<<grid, kBlock, 0, s->stream>>>(g, wall_spec(s), f, dst, nullptr);
        return launched(s, "k_gather");
      case LBL_OBS_RHO:
        k_gather<S, DEV, Q><<<grid, kBlock, 0, s->stream>>>(g, wall_spec(s), f, nullptr, dst);
        return launched(s, "k_gather");
      case LBL_OBS_U: {
        if (s->p.coupling == LBL_SMOL_ONLY) return LBL_E_UNSUPPORTED;
        S* ubuf = static_cast<S*>(s->u);
        const int full = s->p.coupling == LBL_FULL;
        if (full && s->p.force_form == LBL_FORCE_STRESS) {
          if (int rc = stress_force(s, psi)) return rc;
        } else if (full) {
          if (int rc = launch_mu(s, psi, static_cast<S*>(s->mu))) return rc;
        }
        const LBArgs<S> a = lb_args(s, f, nullptr, psi, ubuf, full, 0);
        if (int rc = launch_lb(s, a, false, "k_lb_u")) return rc;
        const int64_t nu = static_cast<int64_t>(s->d) * s->N;
        k_to_f64<S><<<grid_for64(nu), kBlock, 0, s->stream>>>(nu, ubuf, dst);
        return launched(s, "k_to_f64");
      }
      case LBL_OBS_TOTALS:
        return totals(s, dst);
      case LBL_OBS_SK_FULL: {
        if (!s->p.sample_full_k) return LBL_E_UNSUPPORTED;
        const int n = static_cast<int>(half_spectrum(s->p));
        const double inv = 1.0 / static_cast<double>(s->nsamples > 0 ? s->nsamples : 1);
        k_scale<<<grid_for(n), kBlock, 0, s->stream>>>(n, inv, s->fk_acc, dst);
        return launched(s, "k_scale");
      }
      case LBL_OBS_PSIK_AXES:
        return sample(s, false, dst);
      case LBL_OBS_HEIGHTS: {
        const int C = Lat<Q>::D == 3 ? s->p.nx * s->p.ny : s->p.nx;
        const int L = Lat<Q>::D == 3 ? s->p.nz : s->p.ny;
        k_heights<S><<<dim3((C + 255) / 256, 2), 256, 0, s->stream>>>(C, L, psi, dst);
        return launched(s, "k_heights");
      }
      case LBL_OBS_SK_AXES:
      case LBL_OBS_UK_AXES:
      case LBL_OBS_SK2_AXES:
      case LBL_OBS_UK2_AXES: {
        // Accumulators hold the sums of |X|^2/N, then of its square.
        const double inv = 1.0 / static_cast<double>(s->nsamples > 0 ? s->nsamples : 1);
        const bool psi_k = what == LBL_OBS_SK_AXES || what == LBL_OBS_SK2_AXES;
        const bool second = what == LBL_OBS_SK2_AXES || what == LBL_OBS_UK2_AXES;
        const int n = static_cast<int>((psi_k ? 1 : s->d) * s->d * s->Lmax);
        const double* src = (psi_k ? s->sk : s->uk) + (second ? n : 0);
        k_scale<<<grid_for(n), kBlock, 0, s->stream>>>(n, inv, src, dst);
        return launched(s, "k_scale");
      }
      default:
        return LBL_E_UNSUPPORTED;
    }
  }
};

using StepFn = int (*)(lbl_sim*, int64_t);
using InitFn = int (*)(lbl_sim*, const lbl_init*);
using ObsFn = int (*)(lbl_sim*, int, double*);

using TablesFn = void (*)(const std::vector<lbl_sim*>&, int, int, void*, std::vector<Work>&,
                          std::vector<Work>&);
using EnqueueFn = int (*)(hipStream_t, const void*, RepState*, int, const Work*, int, int,
                          const Work*, int, int, bool, int, bool, int64_t);

using ChunkFn = int (*)(lbl_sim*);

struct Table {
  StepFn step;
  InitFn init;
  ChunkFn chunks;
  ObsFn observe;
  TablesFn tables;
  EnqueueFn enqueue;
  size_t replica_bytes;
};

template <typename S, bool DEV, int Q, int SMOL>
Table table_for() {
  using I = Impl<S, DEV, Q, SMOL>;
  return Table{&I::steps, &I::init, &I::default_chunks, &I::observe, &I::tables,
               &I::enqueue_group, I::replica_bytes()};
}

template <typename S, bool DEV>
Table select_lattice(const lbl_params& p) {
  const bool fv = p.smol == LBL_SMOL_FV;
  if (p.lattice == LBL_D2Q9) return fv ? table_for<S, DEV, 9, kFV>() : table_for<S, DEV, 9, kFD>();
  if (p.lattice == LBL_D3Q15)
    return fv ? table_for<S, DEV, 15, kFV>() : table_for<S, DEV, 15, kFD>();
  return fv ? table_for<S, DEV, 19, kFV>() : table_for<S, DEV, 19, kFD>();
}

Table select(const lbl_params& p) {
  if (p.precision == LBL_FP32DEV) return select_lattice<float, true>(p);
  return select_lattice<double, false>(p);
}

// Device allocations of one simulation, in creation order.
constexpr int kPlanBuffers = 23;
using Plan = std::array<size_t, kPlanBuffers>;

Plan alloc_plan(const lbl_params& p) {
  const int q = p.lattice, d = p.lattice == LBL_D2Q9 ? 2 : 3;
  const size_t N = static_cast<size_t>(p.nx) * p.ny * p.nz;
  const size_t sz = p.precision == LBL_FP64 ? 8 : 4;
  const int Lmax = std::max(p.nx, std::max(p.ny, p.nz));
  const int nparts = std::min(1024, std::max(1, static_cast<int>((N + kBlock - 1) / kBlock)));
  return Plan{sz * N * q, sz * N * q, sz * N, sz * N, sz * N, sz * N, sz * N, sz * N,
          sz * N * d, sz * N, sizeof(double) * 10 * nparts, sizeof(double) * 16,
          sizeof(double) * kMaxFields * 3 * Lmax,
          sizeof(double) * kMaxFields * static_cast<size_t>(p.nz) * p.nx,
          sizeof(double) * 2 * d * Lmax, sizeof(double) * 2 * d * d * Lmax, sz * N * d,
          // FD noise in Fourier space: half spectrum (complex) and amplitude table
          p.fd_noise == LBL_FDNOISE_FOURIER ? 2 * sz * half_spectrum(p) : 0,
          p.fd_noise == LBL_FDNOISE_FOURIER ? sz * half_spectrum(p) : 0,
          // force_form STRESS: the stress components (not stored by the fused
          // FV 3-D pass) and the force density
          p.force_form == LBL_FORCE_STRESS && (p.smol != LBL_SMOL_FV || d == 2)
              ? sz * N * d * (d + 1) / 2
              : 0,
          p.force_form == LBL_FORCE_STRESS ? sz * N * d : 0,
          // sample_full_k: the half spectrum of psi and its FP64 accumulator
          p.sample_full_k ? 2 * sz * half_spectrum(p) : 0,
          p.sample_full_k ? sizeof(double) * half_spectrum(p) : 0};
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
    case LBL_OBS_SK2_AXES:
      return 8 * static_cast<size_t>(s->d) * s->Lmax;
    case LBL_OBS_UK_AXES:
    case LBL_OBS_UK2_AXES:
      return 8 * static_cast<size_t>(s->d) * s->d * s->Lmax;
    case LBL_OBS_PSIK_AXES:
      return 8 * 2 * static_cast<size_t>(s->d) * s->Lmax;
    case LBL_OBS_STEP:
    case LBL_OBS_NSAMPLES:
      return 8;
    case LBL_OBS_SK_FULL:
      return s->p.sample_full_k ? 8 * half_spectrum(s->p) : 0;
    case LBL_OBS_HEIGHTS:
      return 8 * 2 * static_cast<size_t>(s->p.nx) * (s->d == 3 ? s->p.ny : 1);
    default:
      return 0;
  }
}

// Fields of a simulation that follow from its parameters alone: sizes, the
// Philox key, the relaxation rates and noise amplitudes of the mode classes,
// and the default launch schedule.
void setup_fields(lbl_sim* s, const lbl_params* params) {
  s->p = *params;
  s->q = params->lattice;
  s->d = params->lattice == LBL_D2Q9 ? 2 : 3;
  s->N = params->nx * params->ny * params->nz;
  s->Lmax = std::max(params->nx, std::max(params->ny, params->nz));
  s->ssize = params->precision == LBL_FP64 ? 8 : 4;
  s->k0 = static_cast<uint32_t>(params->seed);
  s->k1 = static_cast<uint32_t>(params->seed >> 32);
  const double ws = 1.0 / (0.5 + params->eta / (params->rho * kCs2));
  s->gamma_s = 1.0 - ws;
  s->gamma_b = 1.0 - params->omega_bulk;
  s->gamma_g = 1.0 - params->omega_ghost;
  auto sig = [&](double g) { return std::sqrt((1.0 - g * g) * params->rho * params->kT / kCs2); };
  s->sigma_s = sig(s->gamma_s);
  s->sigma_b = sig(s->gamma_b);
  s->sigma_g = sig(s->gamma_g);
  // z-chunks of the tiled SMOL kernels: set from their occupancy at init.
  s->zc = s->zc_prep = s->zc_uend = params->nz;
  // The SMOL noise is drawn in the velocity pass where there is one.
  s->overlap = 3;
  // LB blocks: the widest power of two up to 256 that fits along x (whole
  // rows where possible, so that pulls shifted along x stay inside a block).
  s->lb_lw = 5;
  while (s->lb_lw < 8 && (2 << s->lb_lw) <= params->nx) ++s->lb_lw;
  s->nparts = std::min(1024, std::max(1, grid_for(s->N)));
}

// Buffers of the allocation plan, in plan order.
void assign_buffers(lbl_sim* s, const std::array<void*, kPlanBuffers>& b) {
  s->f[0] = b[0];
  s->f[1] = b[1];
  s->psi[0] = b[2];
  s->psi[1] = b[3];
  s->phi[0] = b[4];
  s->phi[1] = b[5];
  s->acc = b[6];
  s->mu = b[7];
  s->u = b[8];
  s->noise = b[9];
  s->part = static_cast<double*>(b[10]);
  s->tot = static_cast<double*>(b[11]);
  s->planes = static_cast<double*>(b[12]);
  s->col = static_cast<double*>(b[13]);
  s->sk = static_cast<double*>(b[14]);
  s->uk = static_cast<double*>(b[15]);
  s->u_end = b[16];
  s->fspec = b[17];
  s->famp = b[18];
  s->sig = b[19];
  s->fstress = b[20];
  s->fk_spec = b[21];
  s->fk_acc = static_cast<double*>(b[22]);
}

int create_impl(const lbl_params* params, const lbl_init* init, const lbl_env* env,
                lbl_sim** out) {
  if (!out) return fail(nullptr, LBL_E_INVAL, "out must not be NULL");
  *out = nullptr;
  if (int rc = validate(params, init)) return rc;
  lbl_sim* s = new (std::nothrow) lbl_sim();
  if (!s) return fail(nullptr, LBL_E_NOMEM, "host allocation failed");
  setup_fields(s, params);
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
  const size_t N = static_cast<size_t>(s->N);
  const size_t sz = s->ssize;
  const Plan plan = alloc_plan(*params);
  std::array<void*, kPlanBuffers> bufs{};
  bool ok = true;
  for (int k = 0; k < kPlanBuffers; ++k) {
    bufs[k] = dev_alloc(s, plan[k]);
    ok = ok && bufs[k];
  }
  if (ok) assign_buffers(s, bufs);
  if (!ok) {
    std::string msg = "device allocation failed";
    release_all(s);
    delete s;
    return fail(nullptr, LBL_E_NOMEM, msg);
  }
  rc = hip_check(s, hipMemsetAsync(s->noise, 0, sz * N, s->stream), "clear noise");
  if (!rc)
    rc = hip_check(s, hipMemsetAsync(s->sk, 0, sizeof(double) * 2 * s->d * s->Lmax, s->stream),
                   "clear sk");
  if (!rc)
    rc = hip_check(s, hipMemsetAsync(s->uk, 0, sizeof(double) * 2 * s->d * s->d * s->Lmax,
                                     s->stream),
                   "clear uk");
  if (!rc) rc = hip_check(s, hipMemsetAsync(s->u, 0, sz * N * s->d, s->stream), "clear u");
  if (!rc) rc = select(s->p).init(s, init);
  s->step = init->step0;
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

// ---------------------------------------------------------------------------
// Pool.
// ---------------------------------------------------------------------------
double now_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct PoolReq {
  int64_t id = 0;
  lbl_params p{};
  lbl_init init{};
  std::vector<double> user_f, user_psi;
  int64_t nsteps = 0, done_steps = 0;
  int32_t flags = 0;
  int state = LBL_REQ_QUEUED;
  lbl_sim* sim = nullptr;
  uint64_t bytes = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  std::vector<double> totals, sk, psi;
  std::string err;
};

struct GroupKey {
  int precision, lattice, smol, rk, ghost, walls;
  bool operator<(const GroupKey& o) const {
    if (precision != o.precision) return precision < o.precision;
    if (lattice != o.lattice) return lattice < o.lattice;
    if (smol != o.smol) return smol < o.smol;
    if (rk != o.rk) return rk < o.rk;
    if (ghost != o.ghost) return ghost < o.ghost;
    return walls < o.walls;
  }
};

struct DevBuf {
  void* ptr = nullptr;
  size_t cap = 0;
};

struct Group {
  GroupKey key{};
  std::vector<int64_t> members;
  DevBuf reps, states, wlb, wtile;
  int nlb = 0, ntile = 0;
  int lb_lw = 6;  // tile width the LB work table was built with
  int nt = 0;     // populations streamed non-temporally (large groups)
  int lane = 0;   // stream lane this tick of the group runs on
  bool dirty = true;
  hipGraphExec_t exec = nullptr;
  int64_t exec_steps = 0;
};

GroupKey key_of(const lbl_params& p) {
  return GroupKey{p.precision, p.lattice, p.smol, p.rk_stages, p.omega_ghost != 1.0 ? 1 : 0,
                  p.walls == LBL_WALLS_LAST ? 1 : 0};
}

}  // namespace

constexpr int kPoolLanes = 4;  // streams on which groups of different kinds run concurrently

struct lbl_pool {
  uint64_t budget = 0, used = 0;
  lbl_env env{};
  hipStream_t stream = nullptr;           // admission, tables, retirement
  hipStream_t lane[kPoolLanes] = {};      // batched ticks, one lane per group
  int device = 0;
  std::deque<int64_t> queue;
  std::map<int64_t, PoolReq> reqs;
  int64_t next_id = 1;
  std::map<GroupKey, Group> groups;
  int xcd_swizzle = 1;
  int zc_override = 0;
  int lb_lw = 6;  // log2 of the LB tile width of the batched launches
  int64_t ticks = 0, site_updates = 0;
  std::string err;
};

namespace {

void* pool_alloc(lbl_pool* pl, size_t bytes) {
  void* ptr = nullptr;
  if (pl->env.alloc) return pl->env.alloc(pl->env.ctx, bytes, pl->stream);
  return hipMalloc(&ptr, bytes) == hipSuccess ? ptr : nullptr;
}

void pool_free(lbl_pool* pl, void* ptr) {
  if (!ptr) return;
  if (pl->env.free)
    pl->env.free(pl->env.ctx, ptr, pl->stream);
  else
    (void)hipFree(ptr);
}

bool ensure(lbl_pool* pl, DevBuf& b, size_t bytes) {
  if (b.cap >= bytes && b.ptr) return true;
  pool_free(pl, b.ptr);
  b.cap = std::max<size_t>(bytes, 256);
  b.ptr = pool_alloc(pl, b.cap);
  if (!b.ptr) b.cap = 0;
  return b.ptr != nullptr;
}

void drop_graph(Group& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g.exec = nullptr;
  g.exec_steps = 0;
}

// Block b of the launch runs on XCD (b mod 8); give each XCD a contiguous
// range of the work table so that neighbouring tiles share its L2.
void xcd_order(std::vector<Work>& w) {
  const size_t n = w.size();
  if (n < 16) return;
  const size_t q = n / 8, r = n % 8;
  size_t start[8];
  size_t acc = 0;
  for (size_t x = 0; x < 8; ++x) {
    start[x] = acc;
    acc += q + (x < r ? 1 : 0);
  }
  std::vector<Work> out(n);
  for (size_t i = 0; i < n; ++i) out[i] = w[start[i % 8] + i / 8];
  w.swap(out);
}

int pool_fail(lbl_pool* pl, int code, const std::string& msg) {
  pl->err = msg;
  return code;
}

void finish_request(lbl_pool* pl, PoolReq& r, int state) {
  if (r.sim) {
    (void)lbl_destroy(r.sim);
    r.sim = nullptr;
    pl->used -= r.bytes;
  }
  r.state = state;
  r.t_done = now_seconds();
}

// Collect the results of a request that has finished its steps.
void retire(lbl_pool* pl, PoolReq& r) {
  lbl_sim* s = r.sim;
  double t[10];
  int rc = lbl_observe(s, LBL_OBS_TOTALS, t, sizeof(t), 0);
  if (!rc) r.totals.insert(r.totals.end(), t, t + 10);
  // A request whose state became non-finite fails alone: replicas share no
  // memory, so the others are unaffected.
  if (!rc && !std::all_of(t, t + 10, [](double v) { return std::isfinite(v); })) {
    rc = fail(s, LBL_E_NONFINITE, "non-finite state at completion");
  }
  std::vector<double> cur(2 * static_cast<size_t>(s->d) * s->Lmax);
  if (!rc) rc = lbl_observe(s, LBL_OBS_PSIK_AXES, cur.data(), cur.size() * 8, 0);
  if (!rc) {
    r.sk.assign(static_cast<size_t>(s->d) * s->Lmax, 0.0);
    for (size_t k = 0; k < r.sk.size(); ++k)
      r.sk[k] = (cur[2 * k] * cur[2 * k] + cur[2 * k + 1] * cur[2 * k + 1]) / s->N;
  }
  if (!rc && (r.flags & LBL_KEEP_PSI)) {
    r.psi.resize(static_cast<size_t>(s->N));
    rc = lbl_observe(s, LBL_OBS_PSI, r.psi.data(), r.psi.size() * 8, 0);
  }
  if (rc) r.err = s->err;
  finish_request(pl, r, rc ? LBL_REQ_FAILED : LBL_REQ_DONE);
}

int admit(lbl_pool* pl) {
  while (!pl->queue.empty()) {
    PoolReq& r = pl->reqs[pl->queue.front()];
    if (pl->used + r.bytes > pl->budget) break;
    pl->queue.pop_front();
    lbl_init ini = r.init;
    if (ini.kind == LBL_INIT_USER) {
      ini.f0 = r.user_f.data();
      ini.psi0 = r.user_psi.data();
      ini.user_on_device = 0;
    }
    lbl_sim* s = nullptr;
    const int rc = create_impl(&r.p, &ini, &pl->env, &s);
    if (rc) {
      r.err = g_create_error;
      r.state = LBL_REQ_FAILED;
      r.t_done = now_seconds();
      continue;
    }
    r.sim = s;
    pl->used += r.bytes;
    r.state = LBL_REQ_RUNNING;
    r.t_start = now_seconds();
    r.user_f.clear();
    r.user_f.shrink_to_fit();
    r.user_psi.clear();
    r.user_psi.shrink_to_fit();
    double t[10];
    if (lbl_observe(s, LBL_OBS_TOTALS, t, sizeof(t), 0) == LBL_OK)
      r.totals.assign(t, t + 10);
    Group& g = pl->groups[key_of(r.p)];
    g.key = key_of(r.p);
    g.members.push_back(r.id);
    g.dirty = true;
    if (r.nsteps == 0) {
      retire(pl, r);
      g.members.pop_back();
    }
  }
  return LBL_OK;
}

int run_group(lbl_pool* pl, Group& g, int64_t max_steps) {
  if (g.members.empty()) return LBL_OK;
  lbl_sim* first = pl->reqs[g.members.front()].sim;
  const Table t = select(first->p);
  const int n = static_cast<int>(g.members.size());
  if (g.dirty) {
    drop_graph(g);
    std::vector<lbl_sim*> sims;
    std::vector<RepState> st;
    for (int64_t id : g.members) {
      PoolReq& r = pl->reqs[id];
      sims.push_back(r.sim);
      st.push_back(RepState{r.sim->cur, r.sim->pcur, static_cast<uint32_t>(r.sim->step),
                            static_cast<int>(r.nsteps - r.done_steps)});
    }
    std::vector<unsigned char> reps(t.replica_bytes * n);
    std::vector<Work> wlb, wtile;
    t.tables(sims, pl->zc_override, pl->lb_lw, reps.data(), wlb, wtile);
    if (pl->xcd_swizzle) {
      xcd_order(wlb);
      xcd_order(wtile);
    }
    if (!ensure(pl, g.reps, reps.size()) || !ensure(pl, g.states, sizeof(RepState) * n) ||
        !ensure(pl, g.wlb, sizeof(Work) * wlb.size()) ||
        !ensure(pl, g.wtile, sizeof(Work) * wtile.size()))
      return pool_fail(pl, LBL_E_NOMEM, "pool tables: device allocation failed");
    hipError_t e = hipMemcpyAsync(g.reps.ptr, reps.data(), reps.size(), hipMemcpyHostToDevice,
                                  pl->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(g.states.ptr, st.data(), sizeof(RepState) * n, hipMemcpyHostToDevice,
                         pl->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(g.wlb.ptr, wlb.data(), sizeof(Work) * wlb.size(), hipMemcpyHostToDevice,
                         pl->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(g.wtile.ptr, wtile.data(), sizeof(Work) * wtile.size(),
                         hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    if (e != hipSuccess)
      return pool_fail(pl, LBL_E_DEVICE, std::string("pool tables: ") + hipGetErrorString(e));
    g.nlb = static_cast<int>(wlb.size());
    g.lb_lw = pl->lb_lw;
    // Stream the populations past the caches when the group's populations
    // together outgrow the memory-side cache.
    double pop_bytes = 0;
    for (const lbl_sim* m : sims) pop_bytes += 2.0 * m->ssize * m->q * static_cast<double>(m->N);
    g.nt = pop_bytes > kStreamBytes;
    g.ntile = static_cast<int>(wtile.size());
    g.dirty = false;
  }
  int64_t steps = 0;
  for (int64_t id : g.members) {
    const PoolReq& r = pl->reqs[id];
    steps = std::max(steps, r.nsteps - r.done_steps);
  }
  steps = std::min(steps, max_steps);
  if (steps <= 0) return LBL_OK;
  const hipStream_t ls = pl->lane[g.lane];
  if (!g.exec || g.exec_steps != steps) {
    drop_graph(g);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
      return pool_fail(pl, LBL_E_DEVICE, std::string("begin capture: ") + hipGetErrorString(e));
    const int rc = t.enqueue(ls, g.reps.ptr, static_cast<RepState*>(g.states.ptr), n,
                             static_cast<const Work*>(g.wlb.ptr), g.nlb, g.lb_lw,
                             static_cast<const Work*>(g.wtile.ptr), g.ntile, g.key.rk,
                             g.key.ghost != 0, g.nt, g.key.walls != 0, steps);
    e = hipStreamEndCapture(ls, &graph);
    if (rc || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return pool_fail(pl, LBL_E_DEVICE, "graph capture of the batched step failed");
    }
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g.exec = nullptr;
      return pool_fail(pl, LBL_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    g.exec_steps = steps;
  }
  const hipError_t e = hipGraphLaunch(g.exec, ls);
  if (e != hipSuccess)
    return pool_fail(pl, LBL_E_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
  return LBL_OK;
}

// After the tick's graphs have run: copy the device states back into the
// simulations, count the work, retire what is finished.
int settle_group(lbl_pool* pl, Group& g) {
  const int n = static_cast<int>(g.members.size());
  if (n == 0) return LBL_OK;
  std::vector<RepState> st(n);
  hipError_t e = hipMemcpyAsync(st.data(), g.states.ptr, sizeof(RepState) * n,
                                hipMemcpyDeviceToHost, pl->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
  if (e != hipSuccess)
    return pool_fail(pl, LBL_E_DEVICE, std::string("pool states: ") + hipGetErrorString(e));
  std::vector<int64_t> keep;
  for (int i = 0; i < n; ++i) {
    PoolReq& r = pl->reqs[g.members[i]];
    const int64_t done = r.nsteps - st[i].remaining;
    pl->site_updates += (done - r.done_steps) * static_cast<int64_t>(r.sim->N);
    r.done_steps = done;
    r.sim->cur = st[i].cur;
    r.sim->pcur = st[i].pcur;
    r.sim->step = st[i].step;
    if (st[i].remaining <= 0) {
      retire(pl, r);
      g.dirty = true;
    } else {
      keep.push_back(r.id);
    }
  }
  g.members.swap(keep);
  return LBL_OK;
}

int pool_run_impl(lbl_pool* pl, int64_t max_steps, int64_t* pending) {
  if (int rc = hip_check(nullptr, hipSetDevice(pl->device), "hipSetDevice"))
    return pool_fail(pl, rc, g_create_error);
  admit(pl);
  // Admission and table uploads ran on the pool stream; the lanes start after.
  if (int rc = hip_check(nullptr, hipStreamSynchronize(pl->stream), "pool sync"))
    return pool_fail(pl, rc, g_create_error);
  int lane = 0;
  for (auto& kv : pl->groups) {
    if (kv.second.members.empty()) continue;
    kv.second.lane = lane++ % kPoolLanes;
    if (int rc = run_group(pl, kv.second, max_steps)) return rc;
  }
  // Groups of different kinds ran concurrently on their lanes; wait for all
  // before reading the states back and retiring on the pool stream.
  for (hipStream_t ls : pl->lane)
    if (hipStreamSynchronize(ls) != hipSuccess)
      return pool_fail(pl, LBL_E_DEVICE, "pool lane synchronisation failed");
  for (auto& kv : pl->groups)
    if (int rc = settle_group(pl, kv.second)) return rc;
  pl->ticks += 1;
  if (pending) {
    int64_t n = static_cast<int64_t>(pl->queue.size());
    for (auto& kv : pl->groups) n += static_cast<int64_t>(kv.second.members.size());
    *pending = n;
  }
  return LBL_OK;
}

size_t result_bytes(const PoolReq& r, int what) {
  const int d = r.p.lattice == LBL_D2Q9 ? 2 : 3;
  const int Lmax = std::max(r.p.nx, std::max(r.p.ny, r.p.nz));
  switch (what) {
    case LBL_RES_SK_AXES: return 8 * static_cast<size_t>(d) * Lmax;
    case LBL_RES_TOTALS: return 8 * 20;
    case LBL_RES_TIMES: return 8 * 3;
    case LBL_RES_PSI: return 8 * static_cast<size_t>(r.p.nx) * r.p.ny * r.p.nz;
    default: return 0;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Workspace of lbl_step_static: a file-scope device array, one copy per GPU,
// held from the library's load onto that GPU until the process ends.  In host
// code its name is only a stand-in symbol; kernels and copies get the address
// hipGetSymbolAddress returns on each device, resolved once per device.
// ---------------------------------------------------------------------------
__device__ __align__(256) unsigned char scratch[LBL_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of this device's workspace (the device must be current).
int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(nullptr, LBL_E_DEVICE, "device ordinal beyond the workspace table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(nullptr, LBL_E_DEVICE,
                  std::string("hipGetSymbolAddress(workspace): ") + hipGetErrorString(e));
    g_scratch_dev[device] = ptr;
  }
  *out = g_scratch_dev[device];
  return LBL_OK;
}

int zero_async(lbl_sim* s, void* ptr, size_t bytes) {
  const int64_t n = static_cast<int64_t>(bytes / 4);
  if (n == 0) return LBL_OK;
  k_zero_words<<<grid_for64(n), kBlock, 0, s->stream>>>(n, static_cast<uint32_t*>(ptr));
  return hip_check(s, hipGetLastError(), "k_zero_words");
}

int step_static_impl(const lbl_params* params, void* stream, int64_t step0, int64_t nsteps,
                     double* pop, double* psi) {
  if (!params || !pop || !psi)
    return fail(nullptr, LBL_E_INVAL, "params, pop and psi must not be NULL");
  if (nsteps < 0) return fail(nullptr, LBL_E_INVAL, "nsteps must be >= 0");
  lbl_init ini{};
  ini.kind = LBL_INIT_USER;
  ini.user_on_device = 1;
  ini.psi0 = psi;
  ini.f0 = pop;
  ini.step0 = step0;
  if (int rc = validate(params, &ini)) return rc;
  if (params->fd_noise != LBL_FDNOISE_LINK)
    return fail(nullptr, LBL_E_INVAL,
                "the Fourier-space FD noise needs hipFFT plans, which allocate; "
                "not available in lbl_step_static");
  if (params->sample_every != 0 || params->sample_full_k != 0)
    return fail(nullptr, LBL_E_INVAL, "lbl_step_static takes no samples "
                                      "(sample_every and sample_full_k must be 0)");
  // Lay the simulation's buffers out in the workspace, 256-byte aligned.
  const Plan plan = alloc_plan(*params);
  std::array<size_t, kPlanBuffers> off{};
  size_t total = 0;
  for (int k = 0; k < kPlanBuffers; ++k) {
    off[k] = total;
    total += (std::max<size_t>(plan[k], 8) + 255) / 256 * 256;
  }
  if (total > LBL_STATIC_SCRATCH_BYTES)
    return fail(nullptr, LBL_E_NOMEM,
                "the lattice needs " + std::to_string(total) +
                    " bytes of workspace, more than the static workspace of " +
                    std::to_string(static_cast<size_t>(LBL_STATIC_SCRATCH_BYTES)) + " bytes");
  int dev = 0;
  if (int rc = hip_check(nullptr, hipGetDevice(&dev), "hipGetDevice")) return rc;
  void* base = nullptr;
  if (int rc = scratch_address(dev, &base)) return rc;
  std::array<void*, kPlanBuffers> bufs{};
  for (int k = 0; k < kPlanBuffers; ++k) bufs[k] = static_cast<unsigned char*>(base) + off[k];
  lbl_sim s;
  setup_fields(&s, params);
  s.device = dev;
  s.stream = static_cast<hipStream_t>(stream);
  assign_buffers(&s, bufs);
  // The workspace keeps the previous call's contents: clear what the step
  // reads before writing (the SMOL noise stays zero when kT = 0).
  int rc = zero_async(&s, s.noise, s.ssize * static_cast<size_t>(s.N));
  if (!rc) rc = zero_async(&s, s.u, s.ssize * static_cast<size_t>(s.N) * s.d);
  const Table t = select(*params);
  if (!rc) rc = t.init(&s, &ini);
  s.step = step0;
  if (!rc) rc = t.step(&s, nsteps);
  if (!rc) rc = t.observe(&s, LBL_OBS_POP, pop);
  if (!rc) rc = t.observe(&s, LBL_OBS_PSI, psi);
  if (rc) return fail(nullptr, rc, s.err.empty() ? "lbl_step_static failed" : s.err);
  return LBL_OK;
}

}  // namespace

extern "C" {

int lbl_abi_version(void) { return LBL_ABI_VERSION; }

int lbl_step_static(const lbl_params* params, void* stream, int64_t step0, int64_t nsteps,
                    double* pop, double* psi) {
  try {
    g_create_error.clear();
    return step_static_impl(params, stream, step0, nsteps, pop, psi);
  } catch (...) {
    return fail(nullptr, LBL_E_DEVICE, "unexpected exception in lbl_step_static");
  }
}

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
    if (sim->tot_pending) {
      double t[10];
      sim->tot_pending = false;
      int rc = hip_check(sim, hipMemcpyAsync(t, sim->tot, sizeof(t), hipMemcpyDeviceToHost,
                                             sim->stream),
                         "copy sampled totals");
      if (!rc) rc = hip_check(sim, hipStreamSynchronize(sim->stream), "observe sync");
      if (rc) return rc;
      for (int k = 0; k < 10; ++k)
        if (!std::isfinite(t[k]))
          return fail(sim, LBL_E_NONFINITE, "a sampled conserved total is NaN or infinite");
    }
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

int lbl_diag_normals(int32_t device, int32_t precision, uint64_t seed, uint32_t step,
                     uint32_t tag, uint32_t site0, int64_t n_sites, int32_t n_slots,
                     double* dst) {
  if (!dst || n_sites <= 0 || n_sites > (1 << 24) || n_slots <= 0 || n_slots > 64 ||
      (precision != LBL_FP64 && precision != LBL_FP32DEV))
    return LBL_E_INVAL;
  if (hipSetDevice(device) != hipSuccess) return LBL_E_DEVICE;
  const size_t bytes = sizeof(double) * static_cast<size_t>(n_sites) * n_slots;
  double* d = nullptr;
  if (hipMalloc(&d, bytes) != hipSuccess) return LBL_E_NOMEM;
  const int n = static_cast<int>(n_sites);
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  if (precision == LBL_FP64)
    k_diag_normals<double><<<(n + 255) / 256, 256>>>(site0, n, n_slots, step, tag, k0, k1, d);
  else
    k_diag_normals<float><<<(n + 255) / 256, 256>>>(site0, n, n_slots, step, tag, k0, k1, d);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(dst, d, bytes, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  return e == hipSuccess ? LBL_OK : LBL_E_DEVICE;
}

int lbl_set_schedule(lbl_sim* sim, const lbl_schedule* sch) {
  if (!sim || !sch) return LBL_E_INVAL;
  const int w = sch->lb_width;
  int lw = -1;
  for (int k = 5; k <= 8; ++k)
    if (w == (1 << k)) lw = k;
  if (lw < 0) return fail(sim, LBL_E_INVAL, "lb_width must be 32, 64, 128 or 256");
  if (sch->zc < 0 || sch->overlap < 0 || sch->overlap > 3)
    return fail(sim, LBL_E_INVAL, "zc < 0 or overlap not 0, 1, 2 or 3");
  sim->lb_lw = lw;
  sim->lb_swizzle = sch->xcd_swizzle & 3;
  sim->overlap = sch->overlap;
  if (sch->zc > 0) {
    sim->zc = sim->zc_prep = sim->zc_uend = std::min(sch->zc, sim->p.nz);
  } else {
    if (int rc = hip_check(sim, hipSetDevice(sim->device), "hipSetDevice")) return rc;
    if (int rc = select(sim->p).chunks(sim)) return rc;
  }
  return LBL_OK;
}

int lbl_get_schedule(const lbl_sim* sim, lbl_schedule* out) {
  if (!sim || !out) return LBL_E_INVAL;
  out->lb_width = 1 << sim->lb_lw;
  out->xcd_swizzle = sim->lb_swizzle;
  out->zc = sim->zc;
  out->overlap = sim->overlap;
  return LBL_OK;
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
  destroy_aux(sim);
  destroy_events(sim);
  release_all(sim);
  delete sim;
  return LBL_OK;
}

uint64_t lbl_sim_bytes(const lbl_params* params) {
  lbl_init ini{};
  if (!params || validate(params, &ini) != LBL_OK) return 0;
  uint64_t total = 0;
  for (size_t b : alloc_plan(*params)) total += b;
  return total;
}

int lbl_pool_create(uint64_t budget_bytes, const lbl_env* env, lbl_pool** out) {
  if (!out) return LBL_E_INVAL;
  *out = nullptr;
  if (budget_bytes == 0) return fail(nullptr, LBL_E_INVAL, "budget must be > 0");
  if (env && ((env->alloc == nullptr) != (env->free == nullptr)))
    return fail(nullptr, LBL_E_INVAL, "alloc and free must both be set or both NULL");
  lbl_pool* pl = new (std::nothrow) lbl_pool();
  if (!pl) return LBL_E_NOMEM;
  pl->budget = budget_bytes;
  if (env) {
    pl->env = *env;
    pl->device = env->device;
  }
  hipStream_t st = nullptr;
  if (hipSetDevice(pl->device) != hipSuccess ||
      hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    delete pl;
    return fail(nullptr, LBL_E_DEVICE, "pool stream creation failed");
  }
  pl->stream = st;
  pl->env.stream = st;
  for (hipStream_t& ls : pl->lane) {
    if (hipStreamCreateWithFlags(&ls, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : pl->lane)
        if (x) (void)hipStreamDestroy(x);
      (void)hipStreamDestroy(st);
      delete pl;
      return fail(nullptr, LBL_E_DEVICE, "pool stream creation failed");
    }
  }
  *out = pl;
  return LBL_OK;
}

int lbl_pool_submit(lbl_pool* pl, const lbl_params* params, const lbl_init* init, int64_t nsteps,
                    int32_t flags, int64_t* request) {
  if (!pl || !request) return LBL_E_INVAL;
  if (nsteps < 0) return pool_fail(pl, LBL_E_INVAL, "nsteps must be >= 0");
  if (int rc = validate(params, init)) return pool_fail(pl, rc, g_create_error);
  if (params->sample_every != 0)
    return pool_fail(pl, LBL_E_INVAL, "pool requests report the final state (sample_every 0)");
  if (params->fd_noise != LBL_FDNOISE_LINK)
    return pool_fail(pl, LBL_E_INVAL, "Fourier-space FD noise runs in single simulations only");
  if (params->force_form != LBL_FORCE_PSI_GRAD_MU)
    return pool_fail(pl, LBL_E_INVAL, "the stress-divergence force runs in single simulations only");
  if (params->sample_full_k != 0)
    return pool_fail(pl, LBL_E_INVAL, "pool requests report the final state (sample_full_k 0)");
  PoolReq r;
  r.id = pl->next_id++;
  r.p = *params;
  r.init = *init;
  r.nsteps = nsteps;
  r.flags = flags;
  r.t_submit = now_seconds();
  uint64_t bytes = 0;
  for (size_t b : alloc_plan(*params)) bytes += b;
  r.bytes = bytes;
  if (bytes > pl->budget) return pool_fail(pl, LBL_E_NOMEM, "request exceeds the pool budget");
  if (init->kind == LBL_INIT_USER) {
    if (init->user_on_device) return pool_fail(pl, LBL_E_INVAL, "pool USER init must be host data");
    const size_t N = static_cast<size_t>(params->nx) * params->ny * params->nz;
    r.user_f.assign(init->f0, init->f0 + N * params->lattice);
    r.user_psi.assign(init->psi0, init->psi0 + N);
  }
  r.init.f0 = nullptr;
  r.init.psi0 = nullptr;
  *request = r.id;
  pl->queue.push_back(r.id);
  pl->reqs.emplace(r.id, std::move(r));
  return LBL_OK;
}

int lbl_pool_run(lbl_pool* pl, int64_t max_steps, int64_t* pending) {
  if (!pl || max_steps < 0) return LBL_E_INVAL;
  try {
    return pool_run_impl(pl, max_steps, pending);
  } catch (...) {
    return pool_fail(pl, LBL_E_DEVICE, "unexpected exception in lbl_pool_run");
  }
}

int lbl_pool_poll(const lbl_pool* pl, int64_t request, int32_t* state, int64_t* steps_done) {
  if (!pl) return LBL_E_INVAL;
  auto it = pl->reqs.find(request);
  if (it == pl->reqs.end()) return LBL_E_INVAL;
  if (state) *state = it->second.state;
  if (steps_done) *steps_done = it->second.done_steps;
  return LBL_OK;
}

size_t lbl_pool_result_bytes(const lbl_pool* pl, int64_t request, int32_t what) {
  if (!pl) return 0;
  auto it = pl->reqs.find(request);
  return it == pl->reqs.end() ? 0 : result_bytes(it->second, what);
}

int lbl_pool_result(const lbl_pool* pl, int64_t request, int32_t what, void* dst, size_t bytes) {
  if (!pl || !dst) return LBL_E_INVAL;
  auto it = pl->reqs.find(request);
  if (it == pl->reqs.end()) return LBL_E_INVAL;
  const PoolReq& r = it->second;
  const size_t need = result_bytes(r, what);
  if (need == 0) return LBL_E_INVAL;
  if (r.state != LBL_REQ_DONE) return LBL_E_INVAL;
  if (bytes < need) return LBL_E_BUFSIZE;
  double* out = static_cast<double*>(dst);
  switch (what) {
    case LBL_RES_SK_AXES:
      std::copy(r.sk.begin(), r.sk.end(), out);
      return LBL_OK;
    case LBL_RES_TOTALS:
      if (r.totals.size() != 20) return LBL_E_UNSUPPORTED;
      std::copy(r.totals.begin(), r.totals.end(), out);
      return LBL_OK;
    case LBL_RES_TIMES:
      out[0] = r.t_submit;
      out[1] = r.t_start;
      out[2] = r.t_done;
      return LBL_OK;
    case LBL_RES_PSI:
      if (r.psi.empty()) return LBL_E_UNSUPPORTED;
      std::copy(r.psi.begin(), r.psi.end(), out);
      return LBL_OK;
    default:
      return LBL_E_INVAL;
  }
}

int lbl_pool_release(lbl_pool* pl, int64_t request) {
  if (!pl) return LBL_E_INVAL;
  auto it = pl->reqs.find(request);
  if (it == pl->reqs.end()) return LBL_E_INVAL;
  PoolReq& r = it->second;
  if (r.state == LBL_REQ_QUEUED)
    pl->queue.erase(std::remove(pl->queue.begin(), pl->queue.end(), request), pl->queue.end());
  if (r.state == LBL_REQ_RUNNING) {
    Group& g = pl->groups[key_of(r.p)];
    g.members.erase(std::remove(g.members.begin(), g.members.end(), request), g.members.end());
    g.dirty = true;
    drop_graph(g);
    (void)hipStreamSynchronize(pl->stream);
    finish_request(pl, r, LBL_REQ_FAILED);
  }
  pl->reqs.erase(it);
  return LBL_OK;
}

int lbl_pool_stats(const lbl_pool* pl, lbl_pool_info* out) {
  if (!pl || !out) return LBL_E_INVAL;
  *out = lbl_pool_info{};
  out->budget_bytes = pl->budget;
  out->used_bytes = pl->used;
  for (const auto& kv : pl->reqs) {
    const int st = kv.second.state;
    out->queued += st == LBL_REQ_QUEUED;
    out->running += st == LBL_REQ_RUNNING;
    out->done += st == LBL_REQ_DONE;
    out->failed += st == LBL_REQ_FAILED;
  }
  out->ticks = pl->ticks;
  out->site_updates = pl->site_updates;
  return LBL_OK;
}

int lbl_pool_set_schedule(lbl_pool* pl, const lbl_schedule* sch) {
  if (!pl || !sch || sch->zc < 0 || sch->overlap != 0) return LBL_E_INVAL;
  int lw = -1;
  for (int k = 5; k <= 8; ++k)
    if (sch->lb_width == (1 << k)) lw = k;
  if (lw < 0) return LBL_E_INVAL;
  pl->lb_lw = lw;
  pl->xcd_swizzle = sch->xcd_swizzle != 0;
  pl->zc_override = sch->zc;
  for (auto& kv : pl->groups) {
    kv.second.dirty = true;
    drop_graph(kv.second);
  }
  return LBL_OK;
}

int lbl_pool_get_schedule(const lbl_pool* pl, lbl_schedule* out) {
  if (!pl || !out) return LBL_E_INVAL;
  out->lb_width = 1 << pl->lb_lw;
  out->xcd_swizzle = pl->xcd_swizzle;
  out->zc = pl->zc_override;
  out->overlap = 0;
  return LBL_OK;
}

int lbl_pool_destroy(lbl_pool* pl) {
  if (!pl) return LBL_OK;
  (void)hipSetDevice(pl->device);
  for (hipStream_t ls : pl->lane) (void)hipStreamSynchronize(ls);
  (void)hipStreamSynchronize(pl->stream);
  for (auto& kv : pl->reqs)
    if (kv.second.sim) finish_request(pl, kv.second, LBL_REQ_FAILED);
  for (auto& kv : pl->groups) {
    drop_graph(kv.second);
    pool_free(pl, kv.second.reps.ptr);
    pool_free(pl, kv.second.states.ptr);
    pool_free(pl, kv.second.wlb.ptr);
    pool_free(pl, kv.second.wtile.ptr);
  }
  for (hipStream_t ls : pl->lane) (void)hipStreamDestroy(ls);
  (void)hipStreamDestroy(pl->stream);
  delete pl;
  return LBL_OK;
}

const char* lbl_pool_last_error(const lbl_pool* pl) { return pl ? pl->err.c_str() : ""; }

}  // extern "C"
