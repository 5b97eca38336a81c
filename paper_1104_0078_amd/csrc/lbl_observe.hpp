// lbl_observe.hpp -- on-device sampling of the Fourier observables used by
// the paper's checks (Sec. VI): the equal-time structure factor of psi and the
// velocity spectrum at wave vectors on the lattice axes,
//   S_a(k)       = |sum_x psi(x) e^{-i k x_a}|^2 / N,
//   U_{a,b}(k)   = |sum_x u_b(x) e^{-i k x_a}|^2 / N,   k = 2 pi m / L_a,
// accumulated in FP64 over samples together with their squares (for the
// sampling error).  A Fourier mode on an axis only needs the
// plane sums of the field along that axis, so each sample is: plane sums
// (coalesced, fixed-order reductions) and a length-L DFT per axis.  The
// whole-zone spectrum (an option) is a hipFFT transform per sample instead,
// accumulated by k_power_acc.
#pragma once

#include "lbl_device.hpp"

namespace lbl {

constexpr int kMaxFields = 4;  // psi and up to three velocity components
constexpr int kRedBlock = 256;

template <typename S>
struct FieldSet {
  const S* f[kMaxFields];
  int nf;
};

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kRedBlock / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Plane sums over the last axis (z in 3-D, y in 2-D): one block per plane.
// out[(f*3 + axis)*Lmax + h].
template <typename S>
__global__ __launch_bounds__(kRedBlock) void k_plane_last(Geom g, FieldSet<S> fs, int last_axis,
                                                          int Lmax, double* __restrict__ out) {
  __shared__ double red[kRedBlock];
  const int h = blockIdx.x;
  const int count = last_axis == 2 ? g.nx * g.ny : g.nx;
  const size_t base = static_cast<size_t>(h) * count;
  for (int f = 0; f < fs.nf; ++f) {
    double acc = 0.0;
    for (int e = threadIdx.x; e < count; e += kRedBlock) acc += static_cast<double>(fs.f[f][base + e]);
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) out[(f * 3 + last_axis) * Lmax + h] = tot;
  }
}

// 3-D only: plane sums over y = h, one block per plane, rows contiguous in x.
template <typename S>
__global__ __launch_bounds__(kRedBlock) void k_plane_y(Geom g, FieldSet<S> fs, int Lmax,
                                                       double* __restrict__ out) {
  __shared__ double red[kRedBlock];
  const int h = blockIdx.x;
  for (int f = 0; f < fs.nf; ++f) {
    double acc = 0.0;
    for (int z = 0; z < g.nz; ++z) {
      const size_t row = static_cast<size_t>(g.nx) * (h + static_cast<size_t>(g.ny) * z);
      for (int x = threadIdx.x; x < g.nx; x += kRedBlock) acc += static_cast<double>(fs.f[f][row + x]);
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) out[(f * 3 + 1) * Lmax + h] = tot;
  }
}

// Plane sums over x = h in two passes: column sums over y for each (z, x),
// then over z; one thread per x in each pass (coalesced, fixed order).
template <typename S>
__global__ __launch_bounds__(kRedBlock) void k_plane_x1(Geom g, FieldSet<S> fs,
                                                        double* __restrict__ col) {
  const int x = blockIdx.x * kRedBlock + threadIdx.x, z = blockIdx.y;
  if (x >= g.nx) return;
  for (int f = 0; f < fs.nf; ++f) {
    double acc = 0.0;
    for (int y = 0; y < g.ny; ++y)
      acc += static_cast<double>(fs.f[f][x + static_cast<size_t>(g.nx) * (y + static_cast<size_t>(g.ny) * z)]);
    col[(static_cast<size_t>(f) * g.nz + z) * g.nx + x] = acc;
  }
}

__global__ __launch_bounds__(kRedBlock) void k_plane_x2(Geom g, int nf, const double* __restrict__ col,
                                                        int Lmax, double* __restrict__ out) {
  const int x = blockIdx.x * kRedBlock + threadIdx.x;
  if (x >= g.nx) return;
  for (int f = 0; f < nf; ++f) {
    double acc = 0.0;
    for (int z = 0; z < g.nz; ++z) acc += col[(static_cast<size_t>(f) * g.nz + z) * g.nx + x];
    out[(f * 3 + 0) * Lmax + x] = acc;
  }
}

// DFT of the plane sums along each axis.  One thread per (field, axis, m).
// sk[a*Lmax + m] += |X|^2/N for field 0 and sk[(d + a)*Lmax + m] += its
// square; uk[(a*d + b)*Lmax + m] and uk[(d*d + a*d + b)*Lmax + m] likewise
// for field 1 + b; cur (if non-null) receives field 0's complex X as
// [a][m][re,im].
__global__ __launch_bounds__(kRedBlock) void k_axis_dft(Geom g, int d, int nf, int Lmax,
                                                        const double* __restrict__ planes,
                                                        double* __restrict__ sk,
                                                        double* __restrict__ uk,
                                                        double* __restrict__ cur) {
  const int t = blockIdx.x * kRedBlock + threadIdx.x;
  const int m = t % Lmax, a = (t / Lmax) % d, f = t / (Lmax * d);
  if (f >= nf) return;
  const int L = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
  if (m >= L) {  // beyond this axis' length: defined as zero
    if (f == 0 && cur) {
      cur[(a * Lmax + m) * 2 + 0] = 0.0;
      cur[(a * Lmax + m) * 2 + 1] = 0.0;
    }
    return;
  }
  const double* P = planes + (f * 3 + a) * Lmax;
  double re = 0.0, im = 0.0;
  for (int h = 0; h < L; ++h) {
    const long long ph = (static_cast<long long>(m) * h) % L;
    double s, c;
    sincospi(2.0 * static_cast<double>(ph) / static_cast<double>(L), &s, &c);
    re += P[h] * c;
    im -= P[h] * s;
  }
  const double pw = (re * re + im * im) / static_cast<double>(g.N);
  if (f == 0) {
    if (sk) {
      sk[a * Lmax + m] += pw;
      sk[(d + a) * Lmax + m] += pw * pw;
    }
    if (cur) {
      cur[(a * Lmax + m) * 2 + 0] = re;
      cur[(a * Lmax + m) * 2 + 1] = im;
    }
  } else if (uk) {
    uk[(a * d + (f - 1)) * Lmax + m] += pw;
    uk[(d * d + a * d + (f - 1)) * Lmax + m] += pw * pw;
  }
}

__global__ __launch_bounds__(256) void k_scale(int n, double c, const double* __restrict__ in,
                                               double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = c * in[i];
}

// Interface heights along the last axis (Sec. VI.C), one thread per column
// c of C: the zero crossing of psi by linear interpolation between the two
// sites that bracket it, z + psi(z) / (psi(z) - psi(z+1)) at the first z with
// psi(z) psi(z+1) <= 0, in FP64 from the stored values; the window is
// [L/8, 3L/8) for the interface near L/4 (blockIdx.y = 0) and [5L/8, 7L/8)
// for the one near 3L/4; NaN when the window holds no crossing.
// out[k*C + c].
template <typename S>
__global__ __launch_bounds__(256) void k_heights(int C, int L, const S* __restrict__ psi,
                                                 double* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int k = blockIdx.y;
  if (c >= C) return;
  const int lo = k == 0 ? L / 8 : 5 * L / 8, hi = k == 0 ? 3 * L / 8 : 7 * L / 8;
  double h = __builtin_nan("");
  double a = static_cast<double>(psi[c + static_cast<size_t>(C) * lo]);
  for (int z = lo; z < hi; ++z) {
    const double b = static_cast<double>(psi[c + static_cast<size_t>(C) * (z + 1)]);
    if (a * b <= 0.0) {
      h = static_cast<double>(z) + a / (a - b);
      break;
    }
    a = b;
  }
  out[static_cast<size_t>(k) * C + c] = h;
}

}  // namespace lbl
