/*
 * lbl_oracle.h -- interface of the plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference
 * against which the HIP sweep is checked.  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header, table or constant generator with the HIP library.
 *
 * Method: Sumesh, Pagonabarraga & Adhikari, "Lattice Boltzmann - Langevin
 * simulations of binary mixtures" (arXiv:1104.0078): fluctuating lattice
 * Boltzmann (FLBE, Sec. IV and App. B) for momentum, stochastic method of lines
 * (SMOL, Sec. V) for the order parameter psi, marched alternately each step
 * (Sec. VI, opening paragraph).
 *
 * Conventions (lattice units, dx = dt = 1, c_s^2 = 1/3, Sec. VI):
 *   site index s = x + nx*(y + ny*z); 2-D runs have nz = 1.
 *   populations f[i*N + s] in the canonical velocity order of orc_velocities;
 *   vector fields v[alpha*N + s]; scalar fields p[s].
 *   The stored population state at step n is fbar^n, the post-streaming,
 *   pre-collision auxiliary distribution of Eq. (barreln).
 */
#ifndef LBL_ORACLE_H
#define LBL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_D2Q9 = 9, ORC_D3Q15 = 15, ORC_D3Q19 = 19 };
enum { ORC_FD = 0, ORC_FV = 1 };
enum { ORC_FULL = 0, ORC_SMOL_ONLY = 1, ORC_LB_ONLY = 2 };
enum { ORC_TAG_LB = 0, ORC_TAG_SMOL = 1, ORC_TAG_INIT = 2 };
enum { ORC_FDNOISE_LINK = 0, ORC_FDNOISE_FOURIER = 1 };
enum { ORC_FORCE_PSI_GRAD_MU = 0, ORC_FORCE_STRESS = 1 };

typedef struct orc_params {
  int32_t lattice;     /* ORC_D2Q9, ORC_D3Q15 or ORC_D3Q19 */
  int32_t smol;        /* ORC_FD or ORC_FV */
  int32_t coupling;    /* ORC_FULL, ORC_SMOL_ONLY, ORC_LB_ONLY */
  int32_t rk_stages;   /* 1 (Euler), 2 (Heun), 4 (classical RK4) */
  int32_t nx, ny, nz;
  int32_t fd_noise;    /* FD noise construction: ORC_FDNOISE_LINK or ORC_FDNOISE_FOURIER */
  double rho0;         /* mean density, also the density in the noise amplitudes */
  double eta;          /* shear viscosity; shear rate omega_s = 1/(1/2 + eta/(rho0 c_s^2)) */
  double M;            /* mobility */
  double a, b, kappa;  /* Landau coefficients A, B, K of Eq. (feng) and Eq. (Feng) */
  double kT;
  double omega_bulk;   /* relaxation rate of the bulk (trace) stress mode */
  double omega_ghost;  /* relaxation rate of every ghost mode */
  double u_imposed[3]; /* uniform advecting velocity used when coupling == ORC_SMOL_ONLY */
  uint64_t seed;
  int32_t force_form;  /* ORC_FORCE_PSI_GRAD_MU or ORC_FORCE_STRESS */
  int32_t walls;       /* 0: periodic; 1: solid walls across the last axis (below
                          layer 0 and above layer L-1, half a spacing away) */
  double u_wall[6];    /* velocities of the lower wall (0..2) and upper wall (3..5) */
} orc_params;

/* Lattice tables and mode basis. */
int orc_q(int lattice);
int orc_d(int lattice);
void orc_velocities(int lattice, int32_t *c /* q*3 */, double *w /* q */);
void orc_basis(int lattice, double *E /* q*q, E[k*q + i] = e_k(c_i) */);
int orc_nlinks(int lattice);
void orc_links(int lattice, int32_t *c /* nlinks*3 */, double *lambda /* nlinks */);

/* Noise generator (Philox4x32-10 + Box-Muller). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_normal(uint64_t seed, uint32_t site, uint32_t step, uint32_t tag, uint32_t slot);

/* Discrete operators (periodic, or with walls across the last axis: every
 * stencil link that crosses a wall is removed; see orc_laplacian). */
void orc_laplacian(const orc_params *p, const double *in, double *out);
void orc_gradient(const orc_params *p, const double *in, double *out /* d*N */);
void orc_divergence(const orc_params *p, const double *in /* d*N */, double *out);
void orc_chemical_potential(const orc_params *p, const double *psi, double *mu);
void orc_force(const orc_params *p, const double *psi, double *F /* d*N */);
void orc_stress(const orc_params *p, const double *psi, double *sig /* d*d*N */);
void orc_velocity(const orc_params *p, const double *f, const double *F, double *u /* d*N */);

/* Noise fields. */
void orc_fd_noise_divergence(const orc_params *p, const double *zeta /* nlinks*N */, double *out);
void orc_fd_noise_fourier(const orc_params *p, const double *w /* N */, double *out);
void orc_smol_noise(const orc_params *p, uint32_t step, double *out);

/* One site's collision (App. B): fbar (q) -> fstar (q) given force density F
 * (d values) and the normals r (q - d - 1 values, slot order). */
void orc_collide(const orc_params *p, const double *fbar, const double *F,
                 const double *r, double *fstar);

/* SMOL right-hand side G(phi) with frozen velocity u and frozen noise N. */
void orc_smol_rhs(const orc_params *p, const double *phi, const double *u,
                  const double *noise, double *out);

/* Initial state. kind 0: rest + noise, 1: two flat tanh interfaces + noise.
 * boost: uniform initial velocity (3 values, may be NULL). */
int orc_init(const orc_params *p, int kind, double psi_std, const double *boost,
             double *f, double *psi);

/* One coupled step n -> n+1, in place; nsteps consecutive steps from step0. */
int orc_step(const orc_params *p, double *f, double *psi, uint32_t step);
int orc_run(const orc_params *p, double *f, double *psi, uint32_t step0, int64_t nsteps);

/* Totals: [mass, Px, Py, Pz, Psi, L1 mass, L1 Px, L1 Py, L1 Pz, L1 Psi]
 * where P = sum of fbar c (pre-collision momentum). */
void orc_totals(const orc_params *p, const double *f, const double *psi, double *out);

/* Axis structure factors: out[alpha*L_max + k] = |sum_x psi e^{-i k_alpha x_alpha}|^2 / N
 * with k_alpha = 2 pi k / L_alpha, k = 0 .. L_alpha - 1. */
void orc_axis_spectrum(const orc_params *p, const double *field, int32_t lmax, double *out);

/* Interface heights along the last axis (z in 3-D, y in 2-D; length L), per
 * column c (c = x + nx*y in 3-D, x in 2-D; C columns): the zero crossing of
 * psi by linear interpolation between the two sites that bracket it (Sec.
 * VI.C), z + psi(z) / (psi(z) - psi(z+1)) at the first z of the window with
 * psi(z) psi(z+1) <= 0.  Windows: [L/8, 3L/8) for the interface near L/4
 * (out[c]) and [5L/8, 7L/8) for the one near 3L/4 (out[C + c]); NaN if the
 * window holds no crossing. */
void orc_heights(const orc_params *p, const double *psi, double *out);

/* OpenMP threads of the site loops (n > 0), and the current maximum. */
void orc_set_threads(int32_t n);
int32_t orc_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
