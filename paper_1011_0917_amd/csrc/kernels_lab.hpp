// kernels_lab.hpp -- diagnostics of the on-axis laser field: its record in
// the boosted or the lab frame, the Lorentz transform of a record history to
// lab coordinates, and the spatial power spectrum of each record.
#pragma once

#include <math.h>

#include "device_common.hpp"
#include "kernels_particles.hpp"

namespace bfpic {

// Axis row (j = nx/2, k = ny/2), rows 0..nz.  frame 0: E'_y; frame 1: the lab
// field gamma (E'_y - beta B'_x) at the same event, B'_x (stored at half rows:
// row i holds i + 1/2) averaged onto row i.  Periodic z wraps rows -1 and nz.
template <typename R>
__global__ __launch_bounds__(256) void k_axis_record(Geo g, Fields<R> F, int frame, double gb,
                                                     double bb, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > g.nz) return;
  const int j = g.nx / 2, k = g.ny / 2;
  auto at = [&](int r) {
    if (g.periodic_z) r = wrapi(r, g.nz);
    return ((int64_t)(r + kGuard) * g.nx + j) * g.ny + k;
  };
  const double ey = (double)F.F[1][at(i)];
  if (frame == 0) {
    out[i] = ey;
    return;
  }
  const double bx = 0.5 * ((double)F.F[3][at(i - 1)] + (double)F.F[3][at(i)]);
  out[i] = gb * (ey - bb * bx);
}

struct BackK {
  const double* rec;
  const double* tp;  // t' per record, increasing
  const double* z0;  // z' of row 0 per record
  int64_t nrec;
  int n;
  double dz, gamma, beta;
  double t0, dt, zeta0, dzeta, vw;
  int nt, nzeta;
};

// Record r at boosted position z' by linear interpolation; NaN off the rows.
__device__ __forceinline__ double along_record(const BackK& K, int64_t r, double zp) {
  const double u = (zp - K.z0[r]) / K.dz;
  if (!(u >= 0.0 && u <= (double)(K.n - 1))) return NAN;
  int i = (int)floor(u);
  if (i > K.n - 2) i = K.n - 2;
  const double f = u - (double)i;
  const double* x = K.rec + r * K.n;
  return x[i] + f * (x[i + 1] - x[i]);
}

__global__ __launch_bounds__(256) void k_back_transform(BackK K, double* out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)K.nt * K.nzeta) return;
  const int m = (int)(q / K.nzeta), kk = (int)(q - (int64_t)m * K.nzeta);
  const double t = K.t0 + m * K.dt, z = K.zeta0 + kk * K.dzeta + K.vw * t;
  const double tp = K.gamma * (t - K.beta * z), zp = K.gamma * (z - K.beta * t);
  double v = NAN;
  if (tp >= K.tp[0] && tp <= K.tp[K.nrec - 1]) {
    int64_t lo = 0, hi = K.nrec - 1;  // tp[lo] <= t' <= tp[hi]
    while (hi - lo > 1) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (K.tp[mid] <= tp) lo = mid;
      else hi = mid;
    }
    const double a = along_record(K, lo, zp), b = along_record(K, hi, zp);
    v = a + (tp - K.tp[lo]) / (K.tp[hi] - K.tp[lo]) * (b - a);
  }
  out[q] = v;
}

// Power spectrum of one record per workgroup: the record, zero-padded to m
// points, placed in bit-reversed order in LDS, then log2 m radix-2 stages
// (butterflies of span 2 h with twiddle exp(-i pi p / h)), then |X_q|^2.
__global__ __launch_bounds__(256) void k_axis_spectrum(const double* rec, int n, int m, int logm,
                                                       double* out) {
  extern __shared__ double sp[];
  double* re = sp;
  double* im = sp + m;
  const int64_t r = blockIdx.x;
  const double* x = rec + r * n;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const int b = (int)(__brev((unsigned)i) >> (32 - logm));
    re[b] = i < n ? x[i] : 0.0;
    im[b] = 0.0;
  }
  __syncthreads();
  for (int h = 1; h < m; h <<= 1) {
    for (int t = threadIdx.x; t < m / 2; t += blockDim.x) {
      const int p = t & (h - 1);
      const int i0 = ((t - p) << 1) + p, i1 = i0 + h;
      double s, c;
      sincospi(-(double)p / (double)h, &s, &c);
      const double xr = re[i1] * c - im[i1] * s, xi = re[i1] * s + im[i1] * c;
      re[i1] = re[i0] - xr;
      im[i1] = im[i0] - xi;
      re[i0] += xr;
      im[i0] += xi;
    }
    __syncthreads();
  }
  double* o = out + r * (m / 2 + 1);
  for (int q = threadIdx.x; q <= m / 2; q += blockDim.x) o[q] = re[q] * re[q] + im[q] * im[q];
}

}  // namespace bfpic
