/* Host driver for a sanitised build of the oracle: a few coupled steps of
 * every lattice, variant, coupling and stage count on small odd lattices,
 * plus the operators and observables, so that AddressSanitizer and
 * UndefinedBehaviorSanitizer see every code path.  Exit 0 means clean. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "lbl_oracle.h"

static int run_case(int lattice, int smol, int coupling, int rk, int nx, int ny, int nz,
                    int kind) {
  orc_params p = {0};
  p.lattice = lattice;
  p.smol = smol;
  p.coupling = coupling;
  p.rk_stages = rk;
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.rho0 = 1.0;
  p.eta = 0.1;
  p.M = 0.1;
  p.a = kind ? -0.04 : 0.04;
  p.b = kind ? 0.04 : 0.1;
  p.kappa = 0.05;
  p.kT = 1e-5;
  p.omega_bulk = 1.0;
  p.omega_ghost = 1.2;
  p.u_imposed[0] = 0.01;
  p.seed = 99;
  const int q = orc_q(lattice), d = orc_d(lattice);
  const size_t N = (size_t)nx * ny * nz;
  double *f = malloc(sizeof(double) * q * N), *psi = malloc(sizeof(double) * N);
  double *v = malloc(sizeof(double) * d * N), *w = malloc(sizeof(double) * d * N);
  double *s = malloc(sizeof(double) * N), *t = malloc(sizeof(double) * 3 * (nx + ny + nz));
  const double boost[3] = {0.01, -0.02, 0.005};
  int rc = orc_init(&p, kind, 1e-3, boost, f, psi);
  if (!rc) rc = orc_run(&p, f, psi, 0, 3);
  orc_laplacian(&p, psi, s);
  orc_gradient(&p, psi, v);
  orc_divergence(&p, v, s);
  orc_chemical_potential(&p, psi, s);
  orc_force(&p, psi, v);
  orc_velocity(&p, f, v, w);
  orc_smol_noise(&p, 3, s);
  orc_smol_rhs(&p, psi, w, s, s);
  double tot[10];
  orc_totals(&p, f, psi, tot);
  int lmax = nx > ny ? nx : ny;
  if (nz > lmax) lmax = nz;
  orc_axis_spectrum(&p, psi, lmax, t);
  for (int k = 0; k < 10; ++k)
    if (!isfinite(tot[k])) rc = 1;
  free(f);
  free(psi);
  free(v);
  free(w);
  free(s);
  free(t);
  return rc;
}

int main(void) {
  int bad = 0;
  const int rks[3] = {1, 2, 4};
  for (int smol = 0; smol < 2; ++smol)
    for (int cpl = 0; cpl < 3; ++cpl)
      for (int r = 0; r < 3; ++r) {
        bad |= run_case(ORC_D2Q9, smol, cpl, rks[r], 7, 5, 1, cpl == 0);
        bad |= run_case(ORC_D3Q19, smol, cpl, rks[r], 5, 4, 6, cpl == 0);
      }
  printf(bad ? "FAILED\n" : "clean\n");
  return bad;
}
