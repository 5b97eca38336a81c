/*
 * lbl_oracle.c -- plain FP64 CPU oracle of one coupled FLBE + SMOL step.
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
 * CPU-baseline leg are its only users.  It is deliberately slow and literal:
 * every field is materialised, every operator is a plain loop over sites with
 * periodic wrap, the collision is a dense change of basis, and every sum runs
 * in a fixed serial order.  OpenMP only splits independent per-site loops.
 * Compiled with -ffp-contract=off so that no fused multiply-add is formed.
 *
 * Paper: P.T. Sumesh, I. Pagonabarraga, R. Adhikari, arXiv:1104.0078.
 * Readings where the paper is silent, ambiguous or garbled are marked
 * "reading:" below; each is listed, with its justification, in the design
 * notes shipped with the repository.
 */
#include "lbl_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define CS2 (1.0 / 3.0) /* c_s^2 = 1/3 for dx = dt = 1 (Sec. VI) */

/* ------------------------------------------------------------------------ */
/* Lattice tables (Sec. IV, App. B: DdQn velocity sets with weights w_i).   */
/* ------------------------------------------------------------------------ */

static const int32_t C9[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

static const int32_t C19[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W19[19] = {
    1.0 / 3,
    1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* D3Q15, the paper's own lattice (Sec. VI): rest 2/9, the 6 axis links 1/9,
 * the 8 cube corners 1/72; opposite velocities adjacent. */
static const int32_t C15[15][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};
static const double W15[15] = {
    2.0 / 9,
    1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
    1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72};

int orc_q(int lattice) {
  return lattice == ORC_D2Q9 ? 9 : (lattice == ORC_D3Q15 ? 15 : (lattice == ORC_D3Q19 ? 19 : 0));
}
int orc_d(int lattice) {
  return lattice == ORC_D2Q9 ? 2 : ((lattice == ORC_D3Q15 || lattice == ORC_D3Q19) ? 3 : 0);
}

void orc_velocities(int lattice, int32_t *c, double *w) {
  int q = orc_q(lattice);
  for (int i = 0; i < q; i++) {
    for (int a = 0; a < 3; a++)
      c[3 * i + a] = lattice == ORC_D2Q9 ? C9[i][a] : (lattice == ORC_D3Q15 ? C15[i][a] : C19[i][a]);
    w[i] = lattice == ORC_D2Q9 ? W9[i] : (lattice == ORC_D3Q15 ? W15[i] : W19[i]);
  }
}

/* Monomial k evaluated at velocity (x, y, z).  Reading: the mode basis is the
 * Gram-Schmidt orthonormalisation of these monomials under the weighted inner
 * product <a,b> = sum_i w_i a(c_i) b(c_i).  Modes 0..d are mass and momentum,
 * then the stress modes (bulk first, then shear), then the ghosts.  Every
 * 3-D lattice has 6 stress modes (4..9). */
static double monomial(int lattice, int k, double x, double y, double z) {
  if (lattice == ORC_D2Q9) {
    switch (k) {
      case 0: return 1.0;
      case 1: return x;
      case 2: return y;
      case 3: return x * x + y * y;
      case 4: return x * x - y * y;
      case 5: return x * y;
      case 6: return x * y * y;
      case 7: return x * x * y;
      default: return x * x * y * y;
    }
  }
  if (lattice == ORC_D3Q15) {
    /* 1, x, y, z, c^2, x^2, y^2, xy, xz, yz, x c^2, y c^2, z c^2, c^4, xyz */
    double c2 = x * x + y * y + z * z;
    switch (k) {
      case 0: return 1.0;
      case 1: return x;
      case 2: return y;
      case 3: return z;
      case 4: return c2;
      case 5: return x * x;
      case 6: return y * y;
      case 7: return x * y;
      case 8: return x * z;
      case 9: return y * z;
      case 10: return x * c2;
      case 11: return y * c2;
      case 12: return z * c2;
      case 13: return c2 * c2;
      default: return x * y * z;
    }
  }
  switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x + y * y + z * z;
    case 5: return x * x;
    case 6: return y * y;
    case 7: return x * y;
    case 8: return x * z;
    case 9: return y * z;
    case 10: return x * y * y;
    case 11: return x * z * z;
    case 12: return y * x * x;
    case 13: return y * z * z;
    case 14: return z * x * x;
    case 15: return z * y * y;
    case 16: return x * x * y * y;
    case 17: return x * x * z * z;
    default: return y * y * z * z;
  }
}

/* Classical Gram-Schmidt: e_k = normalise(m_k - sum_{l<k} <m_k, e_l> e_l). */
void orc_basis(int lattice, double *E) {
  int q = orc_q(lattice);
  int32_t c[19 * 3];
  double w[19], m[19];
  orc_velocities(lattice, c, w);
  for (int k = 0; k < q; k++) {
    for (int i = 0; i < q; i++)
      m[i] = monomial(lattice, k, c[3 * i], c[3 * i + 1], c[3 * i + 2]);
    double v[19];
    for (int i = 0; i < q; i++) v[i] = m[i];
    for (int l = 0; l < k; l++) {
      double proj = 0.0;
      for (int i = 0; i < q; i++) proj += w[i] * m[i] * E[l * q + i];
      for (int i = 0; i < q; i++) v[i] -= proj * E[l * q + i];
    }
    double nrm = 0.0;
    for (int i = 0; i < q; i++) nrm += w[i] * v[i] * v[i];
    nrm = sqrt(nrm);
    for (int i = 0; i < q; i++) E[k * q + i] = v[i] / nrm;
  }
}

/* Mode classes: 0 mass, 1 momentum, 2 bulk stress, 3 shear stress, 4 ghost. */
static int mode_class(int lattice, int k) {
  int d = orc_d(lattice);
  if (k == 0) return 0;
  if (k <= d) return 1;
  if (k == d + 1) return 2;
  if (lattice == ORC_D2Q9 ? (k <= 5) : (k <= 9)) return 3;
  return 4;
}

/* Undirected links of the Laplacian stencil, one per +/- pair: the offsets
 * whose first non-zero component (x, then y, then z) is +1, ordered by |c|^2
 * and then by descending lexicographic (c_x, c_y, c_z).  lambda is the
 * stencil weight of that neighbour class: 3-D Shinozaki-Oono, Eq. (solap);
 * 2-D (reading): 1/2 nearest, 1/4 diagonal neighbours. */
int orc_nlinks(int lattice) { return lattice == ORC_D2Q9 ? 4 : 13; }

void orc_links(int lattice, int32_t *c, double *lambda) {
  static const int32_t L2[4][3] = {{1, 0, 0}, {0, 1, 0}, {1, 1, 0}, {1, -1, 0}};
  static const int32_t L3[13][3] = {
      {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
      {1, 1, 0}, {1, 0, 1}, {1, 0, -1}, {1, -1, 0}, {0, 1, 1}, {0, 1, -1},
      {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
  int n = orc_nlinks(lattice);
  for (int l = 0; l < n; l++) {
    const int32_t *cc = lattice == ORC_D2Q9 ? L2[l] : L3[l];
    int r2 = 0;
    for (int a = 0; a < 3; a++) {
      c[3 * l + a] = cc[a];
      r2 += cc[a] * cc[a];
    }
    if (lattice == ORC_D2Q9)
      lambda[l] = r2 == 1 ? 0.5 : 0.25;
    else
      lambda[l] = r2 == 1 ? 6.0 / 22.0 : (r2 == 2 ? 3.0 / 22.0 : 1.0 / 22.0);
  }
}

/* ------------------------------------------------------------------------ */
/* Noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) + Box-Muller.   */
/* Reading: the paper fixes only Gaussian white noise with the FDT          */
/* variances of Eqs. (fdt_orderpara), (stressfdt); the generator, its       */
/* counter layout and the Gaussian transform are this project's spec.       */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Normal number of slot `slot`: counter (site, step, slot/4, tag), key = seed;
 * uniforms u_j = (x_j + 1/2) 2^-32; Box-Muller on (u0,u1) -> lanes 0,1 and on
 * (u2,u3) -> lanes 2,3 as sqrt(-2 ln u_even) * {cos, sin}(2 pi u_odd). */
double orc_normal(uint64_t seed, uint32_t site, uint32_t step, uint32_t tag, uint32_t slot) {
  uint32_t ctr[4] = {site, step, slot / 4u, tag};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  int lane = (int)(slot % 4u);
  int even = lane & 2;
  double ue = ((double)out[even] + 0.5) * 0x1p-32;
  double uo = ((double)out[even + 1] + 0.5) * 0x1p-32;
  double r = sqrt(-2.0 * log(ue));
  double t = 2.0 * M_PI * uo;
  return (lane & 1) ? r * sin(t) : r * cos(t);
}

/* ------------------------------------------------------------------------ */
/* Periodic lattice helpers.                                                 */
/* ------------------------------------------------------------------------ */

static int64_t nsites(const orc_params *p) { return (int64_t)p->nx * p->ny * p->nz; }

static int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

/* Site reached from site s by offset (cx, cy, cz). */
static int64_t shift(const orc_params *p, int64_t s, int cx, int cy, int cz) {
  int x = (int)(s % p->nx);
  int y = (int)((s / p->nx) % p->ny);
  int z = (int)(s / ((int64_t)p->nx * p->ny));
  x = wrap(x + cx, p->nx);
  y = wrap(y + cy, p->ny);
  z = wrap(z + cz, p->nz);
  return x + (int64_t)p->nx * (y + (int64_t)p->ny * z);
}

/* Walls (the closing remark of Sec. V.B: the FV scheme admits walls and
 * shear boundaries).  Reading: solid planar walls across the last axis (z in
 * 3-D, y in 2-D), half a lattice spacing below layer 0 and above layer L-1.
 * Every stencil link between a site and a point beyond a wall is removed:
 * there is no flux through a wall.  In a stencil centred at x this means a
 * scalar field takes, beyond the wall, its value at x (the difference along
 * the removed link vanishes), and a flux field takes minus its value at x
 * (the link average of the flux vanishes).  The operators stay adjoint:
 * Div = -Grad^T, and the Laplacians are symmetric with zero row sums. */
static int last_coord(const orc_params *p, int64_t s) {
  if (orc_d(p->lattice) == 3) return (int)(s / ((int64_t)p->nx * p->ny));
  return (int)((s / p->nx) % p->ny);
}

/* 1 when the offset (cx, cy, cz) from site s crosses a wall. */
static int crosses_wall(const orc_params *p, int64_t s, int cx, int cy, int cz) {
  if (!p->walls) return 0;
  int three_d = orc_d(p->lattice) == 3;
  int L = three_d ? p->nz : p->ny;
  int h = last_coord(p, s) + (three_d ? cz : cy);
  (void)cx;
  return h < 0 || h >= L;
}

/* ------------------------------------------------------------------------ */
/* Discrete operators.                                                       */
/* ------------------------------------------------------------------------ */

/* Laplacian L_SO.  3-D: Shinozaki-Oono, Eq. (solap) of App. A:
 *   (6/22) sum N1 + (3/22) sum N2 + (1/22) sum N3 - (80/22) psi.
 * 2-D (reading, the paper gives only 3-D): (1/2) sum N1 + (1/4) sum N2 - 3 psi,
 * with symbol cos qx + cos qy + cos qx cos qy - 3. */
void orc_laplacian(const orc_params *p, const double *in, double *out) {
  int64_t N = nsites(p);
  int three_d = orc_d(p->lattice) == 3;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; s++) {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int zlo = three_d ? -1 : 0, zhi = three_d ? 1 : 0;
    for (int cz = zlo; cz <= zhi; cz++)
      for (int cy = -1; cy <= 1; cy++)
        for (int cx = -1; cx <= 1; cx++) {
          int r2 = cx * cx + cy * cy + cz * cz;
          if (r2 == 0) continue;
          double v = crosses_wall(p, s, cx, cy, cz) ? in[s] : in[shift(p, s, cx, cy, cz)];
          if (r2 == 1) s1 += v;
          else if (r2 == 2) s2 += v;
          else s3 += v;
        }
    if (three_d)
      out[s] = (6.0 / 22.0) * s1 + (3.0 / 22.0) * s2 + (1.0 / 22.0) * s3 - (80.0 / 22.0) * in[s];
    else
      out[s] = 0.5 * s1 + 0.25 * s2 - 3.0 * in[s];
  }
}

/* Gradient.  FD: symmetrised central difference of Sec. IV,
 *   (grad mu)_a(x) = [mu(x + e_a) - mu(x - e_a)] / 2.
 * FV: Eq. (fvgrad), (grad mu)(x) = (1/c_s^2) sum_i w_i c_i mu(x + c_i), the
 * lattice vectors and weights being those of the LB lattice (Sec. V.B). */
void orc_gradient(const orc_params *p, const double *in, double *out) {
  int64_t N = nsites(p);
  int d = orc_d(p->lattice), q = orc_q(p->lattice);
  int32_t c[19 * 3];
  double w[19];
  orc_velocities(p->lattice, c, w);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; s++) {
    for (int a = 0; a < d; a++) {
      double g = 0.0;
      if (p->smol == ORC_FD) {
        int e[3] = {0, 0, 0};
        e[a] = 1;
        double vp = crosses_wall(p, s, e[0], e[1], e[2]) ? in[s]
                                                         : in[shift(p, s, e[0], e[1], e[2])];
        double vm = crosses_wall(p, s, -e[0], -e[1], -e[2])
                        ? in[s]
                        : in[shift(p, s, -e[0], -e[1], -e[2])];
        g = 0.5 * (vp - vm);
      } else {
        for (int i = 0; i < q; i++) {
          int cx = c[3 * i], cy = c[3 * i + 1], cz = c[3 * i + 2];
          double v = crosses_wall(p, s, cx, cy, cz) ? in[s] : in[shift(p, s, cx, cy, cz)];
          g += w[i] * c[3 * i + a] * v;
        }
        g = g / CS2;
      }
      out[a * N + s] = g;
    }
  }
}

/* Divergence of a vector field.  FD: conservative central difference of
 * Sec. V.A, sum_a [X_a(x + e_a) - X_a(x - e_a)] / 2.
 * FV: Gamma . X = (1/c_s^2) sum_i w_i c_i . X(x + c_i).  Reading: this is
 * Eq. (fvdiff) with the symmetric link average of Eqs. (fvflux), (noiseflux)
 * and the normalisation 2/c_s^2 that makes Gamma . Gamma equal Eq. (fvlapft);
 * taken literally Eq. (fvdiff) lacks that factor. */
void orc_divergence(const orc_params *p, const double *in, double *out) {
  int64_t N = nsites(p);
  int d = orc_d(p->lattice), q = orc_q(p->lattice);
  int32_t c[19 * 3];
  double w[19];
  orc_velocities(p->lattice, c, w);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; s++) {
    double div = 0.0;
    if (p->smol == ORC_FD) {
      for (int a = 0; a < d; a++) {
        int e[3] = {0, 0, 0};
        e[a] = 1;
        double vp = crosses_wall(p, s, e[0], e[1], e[2])
                        ? -in[a * N + s]
                        : in[a * N + shift(p, s, e[0], e[1], e[2])];
        double vm = crosses_wall(p, s, -e[0], -e[1], -e[2])
                        ? -in[a * N + s]
                        : in[a * N + shift(p, s, -e[0], -e[1], -e[2])];
        div += 0.5 * (vp - vm);
      }
    } else {
      for (int i = 0; i < q; i++) {
        int cx = c[3 * i], cy = c[3 * i + 1], cz = c[3 * i + 2];
        int out_ = crosses_wall(p, s, cx, cy, cz);
        int64_t t = out_ ? s : shift(p, s, cx, cy, cz);
        double cv = 0.0;
        for (int a = 0; a < d; a++) cv += c[3 * i + a] * (out_ ? -in[a * N + t] : in[a * N + t]);
        div += w[i] * cv;
      }
      div = div / CS2;
    }
    out[s] = div;
  }
}

/* Chemical potential mu = A psi + B psi^3 - K lap psi (Sec. II.A), with the
 * Shinozaki-Oono Laplacian in both variants (Secs. IV, V.A, V.B). */
void orc_chemical_potential(const orc_params *p, const double *psi, double *mu) {
  int64_t N = nsites(p);
  double *lap = (double *)malloc(sizeof(double) * N);
  orc_laplacian(p, psi, lap);
  for (int64_t s = 0; s < N; s++)
    mu[s] = p->a * psi[s] + p->b * psi[s] * psi[s] * psi[s] - p->kappa * lap[s];
  free(lap);
}

/* Force density on the fluid.  Reading: F = -psi grad mu.  The paper writes
 * +psi grad mu, but the tensor it gives (Eq. muf) is the pressure tensor P of
 * the order parameter, whose divergence enters the momentum balance with a
 * minus sign; only the minus sign makes free energy plus kinetic energy
 * non-increasing at kT = 0.  The gradient is the variant's own (Sec. IV for
 * FD; Eq. (fvgrad) for FV). */
/* Order-parameter stress of Eq. (muf), with the variant's own gradient g of
 * psi (orc_gradient) and the Shinozaki-Oono Laplacian:
 *   sigma_ab = K g_a g_b + delta_ab [psi f'(psi) - f - K psi L psi - K/2 |g|^2],
 * f = A psi^2/2 + B psi^4/4, so psi f' - f = A psi^2/2 + 3 B psi^4/4.  Stored
 * as the full d x d tensor, sig[(a*d + b)*N + s]. */
void orc_stress(const orc_params *p, const double *psi, double *sig) {
  int64_t N = nsites(p);
  int d = orc_d(p->lattice);
  double *g = (double *)malloc(sizeof(double) * N * d);
  double *lap = (double *)malloc(sizeof(double) * N);
  orc_gradient(p, psi, g);
  orc_laplacian(p, psi, lap);
  for (int64_t s = 0; s < N; s++) {
    const double ps = psi[s];
    double g2 = 0.0;
    for (int c = 0; c < d; c++) g2 += g[c * N + s] * g[c * N + s];
    const double iso = 0.5 * p->a * ps * ps + 0.75 * p->b * ps * ps * ps * ps -
                       p->kappa * ps * lap[s] - 0.5 * p->kappa * g2;
    for (int a = 0; a < d; a++)
      for (int b = 0; b < d; b++)
        sig[(a * d + b) * N + s] = p->kappa * g[a * N + s] * g[b * N + s] + (a == b ? iso : 0.0);
  }
  free(g);
  free(lap);
}

/* Force density on the fluid.  ORC_FORCE_PSI_GRAD_MU (Sec. IV, the paper's
 * discretisation): F = -psi grad mu with the variant's gradient.
 * ORC_FORCE_STRESS: F_a = -sum_b G_b sigma_ab, the divergence of the stress
 * of Eq. (muf) taken with the same gradient operator; equal to -psi grad mu
 * in the continuum, and its sum over the lattice vanishes exactly for any B
 * (every term is a difference of shifted copies). */
void orc_force(const orc_params *p, const double *psi, double *F) {
  int64_t N = nsites(p);
  int d = orc_d(p->lattice);
  if (p->force_form == ORC_FORCE_STRESS) {
    double *sig = (double *)malloc(sizeof(double) * N * d * d);
    double *gs = (double *)malloc(sizeof(double) * N * d);
    orc_stress(p, psi, sig);
    for (int64_t k = 0; k < N * d; k++) F[k] = 0.0;
    for (int a = 0; a < d; a++) {
      for (int b = 0; b < d; b++) {
        orc_gradient(p, sig + (int64_t)(a * d + b) * N, gs); /* gs[c] = G_c sigma_ab */
        for (int64_t s = 0; s < N; s++) F[a * N + s] -= gs[b * N + s];
      }
    }
    free(sig);
    free(gs);
    return;
  }
  double *mu = (double *)malloc(sizeof(double) * N);
  double *g = (double *)malloc(sizeof(double) * N * d);
  orc_chemical_potential(p, psi, mu);
  orc_gradient(p, mu, g);
  for (int a = 0; a < d; a++)
    for (int64_t s = 0; s < N; s++) F[a * N + s] = -psi[s] * g[a * N + s];
  free(mu);
  free(g);
}

/* Fluid velocity from the auxiliary distribution (App. B):
 * rho = sum fbar, rho u = sum fbar c + F/2 (F a force density, reading). */
void orc_velocity(const orc_params *p, const double *f, const double *F, double *u) {
  int64_t N = nsites(p);
  int d = orc_d(p->lattice), q = orc_q(p->lattice);
  int32_t c[19 * 3];
  double w[19];
  orc_velocities(p->lattice, c, w);
  for (int64_t s = 0; s < N; s++) {
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < q; i++) {
      rho += f[i * N + s];
      for (int a = 0; a < d; a++) j[a] += f[i * N + s] * c[3 * i + a];
    }
    for (int a = 0; a < d; a++) u[a * N + s] = (j[a] + 0.5 * F[a * N + s]) / rho;
  }
}

/* ------------------------------------------------------------------------ */
/* SMOL noise.                                                               */
/* ------------------------------------------------------------------------ */

/* FD noise from link fluxes.  Reading: Sec. V.A builds eta in Fourier space
 * with covariance -2 kT M L(q), Eq. (etafdt).  Here the same Gaussian law is
 * realised in real space: one independent flux zeta_l(x) per undirected link
 * (x, x + c_l) with amplitude sqrt(2 kT M lambda_l), and
 *   N(x) = sum_l A_l [zeta_l(x - c_l) - zeta_l(x)],
 * whose covariance is exactly -2 kT M L_SO because -L_SO is a weighted graph
 * Laplacian with non-negative weights lambda_l. */
void orc_fd_noise_divergence(const orc_params *p, const double *zeta, double *out) {
  int64_t N = nsites(p);
  int nl = orc_nlinks(p->lattice);
  int32_t c[13 * 3];
  double lambda[13];
  orc_links(p->lattice, c, lambda);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; s++) {
    double acc = 0.0;
    for (int l = 0; l < nl; l++) {
      double A = sqrt(2.0 * p->kT * p->M * lambda[l]);
      int64_t back = shift(p, s, -c[3 * l], -c[3 * l + 1], -c[3 * l + 2]);
      acc += A * (zeta[l * N + back] - zeta[l * N + s]);
    }
    out[s] = acc;
  }
}

/* Plain discrete Fourier transform along one axis of a complex field (re,
 * im), every line separately: X(k) = sum_j x(j) exp(sign i 2 pi j k / L),
 * sign -1 forward, +1 inverse (unscaled).  O(L) per output, no fast
 * algorithm: the oracle only runs on small lattices. */
static void dft_axis(const orc_params *p, double *re, double *im, int ax, int sign) {
  const int n[3] = {p->nx, p->ny, p->nz};
  const int L = n[ax];
  if (L == 1) return;
  const int64_t N = nsites(p);
  const int64_t stride = ax == 0 ? 1 : (ax == 1 ? p->nx : (int64_t)p->nx * p->ny);
  const int64_t nlines = N / L;
  double *cs = (double *)malloc(sizeof(double) * L);
  double *sn = (double *)malloc(sizeof(double) * L);
  for (int k = 0; k < L; k++) {
    cs[k] = cos(2.0 * M_PI * k / L);
    sn[k] = sign * sin(2.0 * M_PI * k / L);
  }
#pragma omp parallel
  {
    double *tr = (double *)malloc(sizeof(double) * L);
    double *ti = (double *)malloc(sizeof(double) * L);
#pragma omp for schedule(static)
    for (int64_t line = 0; line < nlines; line++) {
      int64_t base;
      if (ax == 0) base = line * p->nx;
      else if (ax == 1) base = line % p->nx + (line / p->nx) * (int64_t)p->nx * p->ny;
      else base = line;
      for (int k = 0; k < L; k++) {
        double ar = 0.0, ai = 0.0;
        for (int j = 0; j < L; j++) {
          const int m = (int)(((int64_t)j * k) % L);
          const double xr = re[base + j * stride], xi = im[base + j * stride];
          ar += xr * cs[m] - xi * sn[m];
          ai += xr * sn[m] + xi * cs[m];
        }
        tr[k] = ar;
        ti[k] = ai;
      }
      for (int k = 0; k < L; k++) {
        re[base + k * stride] = tr[k];
        im[base + k * stride] = ti[k];
      }
    }
    free(tr);
    free(ti);
  }
  free(cs);
  free(sn);
}

static void dft(const orc_params *p, double *re, double *im, int sign) {
  for (int ax = 0; ax < 3; ax++) dft_axis(p, re, im, ax, sign);
}

/* FD noise built in Fourier space as Sec. V.A states it: eta(q) with
 * covariance -2 kT M L(q) (Eq. etafdt), L the Fourier symbol of the lattice
 * Laplacian (Eq. solapft; its 2-D analogue).  Realisation from a real white
 * field w(x) ~ N(0, 1): N = F^-1[ sqrt(-2 kT M L(q)) F[w] ], whose covariance
 * is the operator -2 kT M L_SO.  L(q) is taken as the transform of the
 * Laplacian stencil itself (orc_laplacian applied to a unit impulse). */
void orc_fd_noise_fourier(const orc_params *p, const double *w, double *out) {
  const int64_t N = nsites(p);
  double *re = (double *)calloc(N, sizeof(double));
  double *im = (double *)calloc(N, sizeof(double));
  double *lr = (double *)calloc(N, sizeof(double));
  double *li = (double *)calloc(N, sizeof(double));
  double *delta = (double *)calloc(N, sizeof(double));
  for (int64_t s = 0; s < N; s++) re[s] = w[s];
  delta[0] = 1.0;
  orc_laplacian(p, delta, lr);
  dft(p, lr, li, -1);  /* L(q), real up to rounding (symmetric stencil) */
  dft(p, re, im, -1);
  for (int64_t s = 0; s < N; s++) {
    const double v = -2.0 * p->kT * p->M * lr[s];
    const double A = v > 0.0 ? sqrt(v) : 0.0;
    re[s] *= A;
    im[s] *= A;
  }
  dft(p, re, im, +1);
  for (int64_t s = 0; s < N; s++) out[s] = re[s] / (double)N;
  free(re);
  free(im);
  free(lr);
  free(li);
  free(delta);
}

/* The noise term N^n of the SMOL right-hand side at step n, frozen over the
 * Runge-Kutta stages (Sec. V).  FD: link fluxes above, zeta_l(x) = normal
 * slot l, or (fd_noise == ORC_FDNOISE_FOURIER) the Fourier construction
 * above with w(x) = normal slot 0.  FV: Eqs. (fvdiff), (noiseflux): node noise xi(x) with covariance
 * 2 kT M delta (Eq. fdt_orderpara), xi_a = sqrt(2 kT M) normal slot a, and
 * N = Gamma . xi. */
void orc_smol_noise(const orc_params *p, uint32_t step, double *out) {
  int64_t N = nsites(p);
  int d = orc_d(p->lattice);
  if (p->smol == ORC_FD && p->fd_noise == ORC_FDNOISE_FOURIER) {
    /* white field: normal slot 0 of each site */
    double *w = (double *)malloc(sizeof(double) * N);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; s++)
      w[s] = orc_normal(p->seed, (uint32_t)s, step, ORC_TAG_SMOL, 0);
    orc_fd_noise_fourier(p, w, out);
    free(w);
  } else if (p->smol == ORC_FD) {
    int nl = orc_nlinks(p->lattice);
    double *zeta = (double *)malloc(sizeof(double) * N * nl);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; s++)
      for (int l = 0; l < nl; l++)
        zeta[l * N + s] = orc_normal(p->seed, (uint32_t)s, step, ORC_TAG_SMOL, (uint32_t)l);
    orc_fd_noise_divergence(p, zeta, out);
    free(zeta);
  } else {
    double *xi = (double *)malloc(sizeof(double) * N * d);
    double amp = sqrt(2.0 * p->kT * p->M);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; s++)
      for (int a = 0; a < d; a++)
        xi[a * N + s] = amp * orc_normal(p->seed, (uint32_t)s, step, ORC_TAG_SMOL, (uint32_t)a);
    orc_divergence(p, xi, out);
    free(xi);
  }
}

/* ------------------------------------------------------------------------ */
/* SMOL right-hand side (Sec. V).                                            */
/* ------------------------------------------------------------------------ */

/* G(phi) = -Div(u phi) + M Div(grad mu(phi)) + N, with u and N frozen.
 * FD (Sec. V.A): Div is the central divergence and the diffusion term is
 * M L_SO mu, the same Shinozaki-Oono stencil as in mu.
 * FV (Sec. V.B, Eq. fvft): Div = Gamma . and the diffusion term is
 * M Gamma . (Gamma mu). */
void orc_smol_rhs(const orc_params *p, const double *phi, const double *u,
                  const double *noise, double *out) {
  int64_t N = nsites(p);
  int d = orc_d(p->lattice);
  double *mu = (double *)malloc(sizeof(double) * N);
  double *flux = (double *)malloc(sizeof(double) * N * d);
  double *adv = (double *)malloc(sizeof(double) * N);
  double *diff = (double *)malloc(sizeof(double) * N);
  orc_chemical_potential(p, phi, mu);
  for (int a = 0; a < d; a++)
    for (int64_t s = 0; s < N; s++) flux[a * N + s] = u[a * N + s] * phi[s];
  orc_divergence(p, flux, adv);
  if (p->smol == ORC_FD) {
    orc_laplacian(p, mu, diff);
  } else {
    orc_gradient(p, mu, flux);
    orc_divergence(p, flux, diff);
  }
  for (int64_t s = 0; s < N; s++) out[s] = -adv[s] + p->M * diff[s] + noise[s];
  free(mu);
  free(flux);
  free(adv);
  free(diff);
}

/* ------------------------------------------------------------------------ */
/* FLBE collision (App. B).                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
  int q, d;
  int32_t c[19 * 3];
  double w[19];
  double E[19 * 19];
  int opp[19];      /* index of the opposite velocity */
  double gamma[19]; /* per-mode gamma_k = 1 - omega_k */
  double sigma[19]; /* per-mode noise amplitude */
} lb_tables;

static double omega_shear(const orc_params *p) {
  /* tau_LB = 1/2 + eta/(rho0 c_s^2): the paper's tau plus dt/2 (Eq. bab uses
   * dt/(tau + dt/2)). */
  return 1.0 / (0.5 + p->eta / (p->rho0 * CS2));
}

static void lb_setup(const orc_params *p, lb_tables *t) {
  t->q = orc_q(p->lattice);
  t->d = orc_d(p->lattice);
  orc_velocities(p->lattice, t->c, t->w);
  orc_basis(p->lattice, t->E);
  for (int i = 0; i < t->q; i++)
    for (int j = 0; j < t->q; j++)
      if (t->c[3 * j] == -t->c[3 * i] && t->c[3 * j + 1] == -t->c[3 * i + 1] &&
          t->c[3 * j + 2] == -t->c[3 * i + 2])
        t->opp[i] = j;
  double ws = omega_shear(p);
  for (int k = 0; k < t->q; k++) {
    int cls = mode_class(p->lattice, k);
    double om = cls == 2 ? p->omega_bulk : (cls == 3 ? ws : p->omega_ghost);
    t->gamma[k] = cls <= 1 ? 0.0 : 1.0 - om;
    /* Equipartition of every non-conserved mode: <m_k^2> = rho0 kT / c_s^2
     * requires sigma_k^2 = (1 - gamma_k^2) rho0 kT / c_s^2 (Secs. III, IV:
     * noise on all dissipative modes, ghosts included). */
    t->sigma[k] = cls <= 1 ? 0.0
                           : sqrt((1.0 - t->gamma[k] * t->gamma[k]) * p->rho0 * p->kT / CS2);
  }
}

/* Post-collision auxiliary distribution in the orthonormal mode basis.  With
 * all rates equal and kT = 0 this is the single-relaxation update below
 * Eq. (barlin); with the ghosts projected out it is Eq. (bab):
 *   fbar*_i = w_i (rho + A.c_i / c_s^2 + B:Q_i / (2 c_s^4)),
 *   A = sum fbar c + F,
 *   B = S + omega (-S + rho u u + tau (u F + F u) + noise stress),
 * generalised to separate bulk, shear and ghost rates (multiple relaxation
 * times) with Landau-Lifshitz noise on every non-conserved mode. */
static void collide_site(const lb_tables *t, const double *fbar, const double *F,
                         const double *r, double *fstar) {
  int q = t->q, d = t->d;
  double cs = sqrt(CS2);
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, u[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < q; i++) {
    rho += fbar[i];
    for (int a = 0; a < d; a++) j[a] += fbar[i] * t->c[3 * i + a];
  }
  for (int a = 0; a < d; a++) u[a] = (j[a] + 0.5 * F[a]) / rho;
  double usq = 0.0, uF = 0.0;
  for (int a = 0; a < d; a++) {
    usq += u[a] * u[a];
    uF += u[a] * F[a];
  }
  /* Second-order equilibrium and the Guo/Nash second-moment source
   * w_i (u F + F u):Q_i / (2 c_s^4). */
  double feq[19], src[19];
  for (int i = 0; i < q; i++) {
    double cu = 0.0, cF = 0.0;
    for (int a = 0; a < d; a++) {
      cu += t->c[3 * i + a] * u[a];
      cF += t->c[3 * i + a] * F[a];
    }
    feq[i] = t->w[i] * rho *
             (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - usq / (2.0 * CS2));
    src[i] = t->w[i] * (cu * cF - CS2 * uF) / (CS2 * CS2);
  }
  double m[19] = {0}, meq[19] = {0}, sk[19] = {0}, mstar[19] = {0};
  for (int k = 0; k < q; k++) {
    for (int i = 0; i < q; i++) {
      m[k] += t->E[k * q + i] * fbar[i];
      meq[k] += t->E[k * q + i] * feq[i];
      sk[k] += t->E[k * q + i] * src[i];
    }
  }
  mstar[0] = m[0];
  for (int a = 0; a < d; a++) mstar[1 + a] = (j[a] + F[a]) / cs;
  for (int k = d + 1; k < q; k++) {
    double g = t->gamma[k];
    mstar[k] = meq[k] + g * (m[k] - meq[k]) + 0.5 * (1.0 + g) * sk[k] +
               t->sigma[k] * r[k - d - 1];
  }
  for (int i = 0; i < q; i++) {
    double v = 0.0;
    for (int k = 0; k < q; k++) v += t->E[k * q + i] * mstar[k];
    fstar[i] = t->w[i] * v;
  }
}

void orc_collide(const orc_params *p, const double *fbar, const double *F,
                 const double *r, double *fstar) {
  lb_tables t;
  lb_setup(p, &t);
  collide_site(&t, fbar, F, r, fstar);
}

/* ------------------------------------------------------------------------ */
/* Initial state.                                                            */
/* ------------------------------------------------------------------------ */

int orc_init(const orc_params *p, int kind, double psi_std, const double *boost,
             double *f, double *psi) {
  int64_t N = nsites(p);
  int q = orc_q(p->lattice), d = orc_d(p->lattice);
  int32_t c[19 * 3];
  double w[19], U[3] = {0.0, 0.0, 0.0};
  orc_velocities(p->lattice, c, w);
  if (boost)
    for (int a = 0; a < d; a++) U[a] = boost[a];
  double usq = 0.0;
  for (int a = 0; a < d; a++) usq += U[a] * U[a];
  /* fbar^0 = second-order equilibrium at density rho0 and velocity U. */
  for (int i = 0; i < q; i++) {
    double cu = 0.0;
    for (int a = 0; a < d; a++) cu += c[3 * i + a] * U[a];
    double fe = w[i] * p->rho0 *
                (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - usq / (2.0 * CS2));
    for (int64_t s = 0; s < N; s++) f[i * N + s] = fe;
  }
  double psi_eq = 0.0, l = 1.0;
  if (kind == 1) {
    if (!(p->a < 0.0 && p->b > 0.0 && p->kappa > 0.0)) return -1;
    /* Eqs. (tanh), (intthick) with A -> |A| (reading). */
    psi_eq = sqrt(-p->a / p->b);
    l = sqrt(-2.0 * p->kappa / p->a);
  }
  int Lh = d == 3 ? p->nz : p->ny;
  for (int64_t s = 0; s < N; s++) {
    double v = psi_std * orc_normal(p->seed, (uint32_t)s, 0u, ORC_TAG_INIT, 0u);
    if (kind == 1) {
      /* Reading: two interfaces at h = L/4 and 3L/4 along the last axis so
       * that the profile is periodic; psi > 0 between them. */
      int h = d == 3 ? (int)(s / ((int64_t)p->nx * p->ny)) : (int)((s / p->nx) % p->ny);
      v += psi_eq * (tanh((h - 0.25 * Lh) / l) - tanh((h - 0.75 * Lh) / l) - 1.0);
    }
    psi[s] = v;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* One coupled step (Sec. VI: FLBE and SMOL marched alternately).            */
/* Reading: both solvers advance from the time-n fields: F^n, u^n and mu^n   */
/* are all computed from (fbar^n, psi^n).                                     */
/* ------------------------------------------------------------------------ */

int orc_step(const orc_params *p, double *f, double *psi, uint32_t step) {
  int64_t N = nsites(p);
  int q = orc_q(p->lattice), d = orc_d(p->lattice);
  if (q == 0) return -1;
  double *F = (double *)calloc((size_t)N * d, sizeof(double));
  double *u = (double *)malloc(sizeof(double) * N * d);

  /* 1-3: mu^n, grad mu^n and the force density F^n. */
  if (p->coupling == ORC_FULL) orc_force(p, psi, F);

  /* 4: velocity u^n (App. B moment relations), or the imposed flow. */
  if (p->coupling == ORC_SMOL_ONLY) {
    for (int a = 0; a < d; a++)
      for (int64_t s = 0; s < N; s++) u[a * N + s] = p->u_imposed[a];
  } else {
    orc_velocity(p, f, F, u);
  }

  /* 5-6: collision, then propagation fbar^{n+1}(x + c_i) = fbar*_i(x). */
  if (p->coupling != ORC_SMOL_ONLY) {
    lb_tables t;
    lb_setup(p, &t);
    double *fn = (double *)malloc(sizeof(double) * N * q);
    int nr = q - d - 1;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; s++) {
      double fb[19], fs[19], Fs[3] = {0.0, 0.0, 0.0}, r[16];
      for (int i = 0; i < q; i++) fb[i] = f[i * N + s];
      for (int a = 0; a < d; a++) Fs[a] = F[a * N + s];
      for (int k = 0; k < nr; k++)
        r[k] = orc_normal(p->seed, (uint32_t)s, step, ORC_TAG_LB, (uint32_t)k);
      collide_site(&t, fb, Fs, r, fs);
      for (int i = 0; i < q; i++) {
        int cx = t.c[3 * i], cy = t.c[3 * i + 1], cz = t.c[3 * i + 2];
        if (crosses_wall(p, s, cx, cy, cz)) {
          /* Halfway bounce-back at a wall moving with velocity U (Ladd):
           * the population returns to s reversed, less 2 w_i rho0 c_i.U/c_s^2. */
          const double *U = last_coord(p, s) == 0 ? p->u_wall : p->u_wall + 3;
          double cU = 0.0;
          for (int a = 0; a < d; a++) cU += t.c[3 * i + a] * U[a];
          fn[t.opp[i] * N + s] = fs[i] - 2.0 * t.w[i] * p->rho0 * cU / CS2;
        } else {
          fn[i * N + shift(p, s, cx, cy, cz)] = fs[i];
        }
      }
    }
    memcpy(f, fn, sizeof(double) * N * q);
    free(fn);
  }

  /* 7: SMOL Runge-Kutta with the noise held constant through the step (Sec. V,
   * Wilkie's scheme).  Reading: only the noise is frozen; each stage sees the
   * advecting velocity of its own time level: u^n at t_n, and at t_{n+1} the
   * velocity of the streamed populations, (jbar^{n+1} + F^n/2)/rho^{n+1} (the
   * time-n force is the only one known before psi^{n+1}); RK4's mid stages use
   * the average of the two.  Freezing u^n over both stages instead leaves the
   * longitudinal momentum at the axis Nyquist wave number, which streaming flips
   * each step and collision never damps, driving the interfaces with one sign
   * through the whole step: two-phase runs then diverge after ~10^3 steps.
   * Default stages: Heun; Euler and classical RK4 are selectable. */
  if (p->coupling != ORC_LB_ONLY) {
    double *noise = (double *)malloc(sizeof(double) * N);
    double *k1 = (double *)malloc(sizeof(double) * N);
    double *k2 = (double *)malloc(sizeof(double) * N);
    double *tmp = (double *)malloc(sizeof(double) * N);
    double *u1 = (double *)malloc(sizeof(double) * N * d);
    double *uh = (double *)malloc(sizeof(double) * N * d);
    if (p->coupling == ORC_FULL) {
      orc_velocity(p, f, F, u1); /* f now holds fbar^{n+1} */
    } else {
      memcpy(u1, u, sizeof(double) * N * d); /* imposed uniform flow */
    }
    for (int64_t k = 0; k < N * d; k++) uh[k] = 0.5 * (u[k] + u1[k]);
    orc_smol_noise(p, step, noise);
    orc_smol_rhs(p, psi, u, noise, k1);
    if (p->rk_stages == 1) {
      for (int64_t s = 0; s < N; s++) psi[s] = psi[s] + k1[s];
    } else if (p->rk_stages == 2) {
      for (int64_t s = 0; s < N; s++) tmp[s] = psi[s] + k1[s];
      orc_smol_rhs(p, tmp, u1, noise, k2);
      for (int64_t s = 0; s < N; s++) psi[s] = psi[s] + 0.5 * (k1[s] + k2[s]);
    } else {
      double *k3 = (double *)malloc(sizeof(double) * N);
      double *k4 = (double *)malloc(sizeof(double) * N);
      for (int64_t s = 0; s < N; s++) tmp[s] = psi[s] + 0.5 * k1[s];
      orc_smol_rhs(p, tmp, uh, noise, k2);
      for (int64_t s = 0; s < N; s++) tmp[s] = psi[s] + 0.5 * k2[s];
      orc_smol_rhs(p, tmp, uh, noise, k3);
      for (int64_t s = 0; s < N; s++) tmp[s] = psi[s] + k3[s];
      orc_smol_rhs(p, tmp, u1, noise, k4);
      for (int64_t s = 0; s < N; s++)
        psi[s] = psi[s] + (k1[s] + 2.0 * k2[s] + 2.0 * k3[s] + k4[s]) / 6.0;
      free(k3);
      free(k4);
    }
    free(noise);
    free(k1);
    free(k2);
    free(tmp);
    free(u1);
    free(uh);
  }
  free(F);
  free(u);
  return 0;
}

int orc_run(const orc_params *p, double *f, double *psi, uint32_t step0, int64_t nsteps) {
  for (int64_t n = 0; n < nsteps; n++) {
    int rc = orc_step(p, f, psi, step0 + (uint32_t)n);
    if (rc) return rc;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Observables.                                                              */
/* ------------------------------------------------------------------------ */

void orc_totals(const orc_params *p, const double *f, const double *psi, double *out) {
  int64_t N = nsites(p);
  int q = orc_q(p->lattice), d = orc_d(p->lattice);
  int32_t c[19 * 3];
  double w[19];
  orc_velocities(p->lattice, c, w);
  for (int k = 0; k < 10; k++) out[k] = 0.0;
  for (int64_t s = 0; s < N; s++) {
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < q; i++) {
      rho += f[i * N + s];
      for (int a = 0; a < d; a++) j[a] += f[i * N + s] * c[3 * i + a];
    }
    out[0] += rho;
    out[5] += fabs(rho);
    for (int a = 0; a < 3; a++) {
      out[1 + a] += j[a];
      out[6 + a] += fabs(j[a]);
    }
    out[4] += psi[s];
    out[9] += fabs(psi[s]);
  }
}

/* Plain DFT of the plane sums along each axis: the structure factor
 * |psi~(q)|^2 / N at q on the axes (Eqs. test1, test2). */
void orc_axis_spectrum(const orc_params *p, const double *field, int32_t lmax, double *out) {
  int64_t N = nsites(p);
  int d = orc_d(p->lattice);
  int L[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < d; a++) {
    double *plane = (double *)calloc((size_t)L[a], sizeof(double));
    for (int64_t s = 0; s < N; s++) {
      int x = (int)(s % p->nx);
      int y = (int)((s / p->nx) % p->ny);
      int z = (int)(s / ((int64_t)p->nx * p->ny));
      int h = a == 0 ? x : (a == 1 ? y : z);
      plane[h] += field[s];
    }
    for (int k = 0; k < lmax; k++) {
      if (k >= L[a]) {
        out[a * lmax + k] = 0.0;
        continue;
      }
      double re = 0.0, im = 0.0;
      for (int h = 0; h < L[a]; h++) {
        double ph = 2.0 * M_PI * (double)k * (double)h / (double)L[a];
        re += plane[h] * cos(ph);
        im -= plane[h] * sin(ph);
      }
      out[a * lmax + k] = (re * re + im * im) / (double)N;
    }
    free(plane);
  }
}

/* Interface heights (Sec. VI.C): zero crossing of psi along the last axis in
 * the two windows around L/4 and 3L/4, by linear interpolation. */
void orc_heights(const orc_params *p, const double *psi, double *out) {
  int d = orc_d(p->lattice);
  int64_t L = d == 3 ? p->nz : p->ny;
  int64_t C = d == 3 ? (int64_t)p->nx * p->ny : p->nx;
  int64_t lo[2] = {L / 8, 5 * L / 8}, hi[2] = {3 * L / 8, 7 * L / 8};
  for (int k = 0; k < 2; k++) {
    for (int64_t c = 0; c < C; c++) {
      double h = NAN;
      for (int64_t z = lo[k]; z < hi[k]; z++) {
        double a = psi[c + C * z], b = psi[c + C * (z + 1)];
        if (a * b <= 0.0) {
          h = (double)z + a / (a - b);
          break;
        }
      }
      out[k * C + c] = h;
    }
  }
}

/* Thread count of the OpenMP site loops (test infrastructure: the CPU
 * baseline times the oracle at one thread and at all host threads). */
void orc_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int32_t orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
