// kernels_diag.hpp -- FP64 diagnostics: field and kinetic energies, charge,
// live count, non-finite flag, on-axis Ez lineout, Gauss residual.
#pragma once

#include "device_common.hpp"
#include "kernels_fields.hpp"
#include "kernels_particles.hpp"

namespace bfpic {

constexpr int kDiagBlock = 256;
constexpr int kDiagMaxBlocks = 512;

// p[0..n) = 0 (a fill kernel rather than a memset node).
__global__ __launch_bounds__(256) void k_zero_f64(double* p, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x)
    p[q] = 0.0;
}

template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* sh) {
  // sh: N * kDiagBlock doubles
  for (int a = 0; a < N; a++) sh[a * kDiagBlock + threadIdx.x] = v[a];
  __syncthreads();
  for (int s = kDiagBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int a = 0; a < N; a++) sh[a * kDiagBlock + threadIdx.x] += sh[a * kDiagBlock + threadIdx.x + s];
    __syncthreads();
  }
  for (int a = 0; a < N; a++) v[a] = sh[a * kDiagBlock];
  __syncthreads();
}

// partial[b * 2 + 0/1] = sum E^2 / sum B^2 of block b over the domain nodes.
template <typename R>
__global__ __launch_bounds__(kDiagBlock) void k_diag_fields(Geo g, Fields<R> F, double* partial,
                                                             int* nanflag) {
  __shared__ double sh[2 * kDiagBlock];
  double v[2] = {0.0, 0.0};
  int bad = 0;
  int64_t total = (int64_t)(g.nz + 1) * g.plane;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(q / g.plane);
    int64_t n = (int64_t)(i + kGuard) * g.plane + (q - (int64_t)i * g.plane);
    for (int c = 0; c < 6; c++) {
      if (!in_domain(g, half_z_eb(c), i)) continue;
      double x = (double)F.F[c][n];
      if (!isfinite(x)) bad = 1;
      v[c < 3 ? 0 : 1] += x * x;
    }
  }
  if (bad) atomicOr(nanflag, 1);
  block_sum<2>(v, sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x * 2 + 0] = v[0];
    partial[blockIdx.x * 2 + 1] = v[1];
  }
}

// partial[b * 4 + ...] = sum w (gamma - 1), sum w (gamma - gamma_b), sum q w, live count.
template <typename R, int DIM>
__global__ __launch_bounds__(kDiagBlock) void k_diag_particles(PSoA<R> S, const int* counts,
                                                                double ub, double gb,
                                                                double* partial, int* nanflag) {
  __shared__ double sh[4 * kDiagBlock];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  int bad = 0;
  int n = counts[0];
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    if (S.id[p] < 0) continue;
    double dx = S.du[0][p], dy = S.du[1][p], dz = S.du[2][p];
    double w = S.w[p];
    double c = 2.0 * ub * dz + (dx * dx + dy * dy + dz * dz);
    double dg = c / (gb + sqrt(gb * gb + c));
    if (!isfinite(dg) || !isfinite((double)S.xi[0][p]) || !isfinite((double)S.xi[1][p])) bad = 1;
    v[0] += w * ((gb - 1.0) + dg);
    v[1] += w * dg;
    v[2] += -w;
    v[3] += 1.0;
  }
  if (bad) atomicOr(nanflag, 1);
  block_sum<4>(v, sh);
  if (threadIdx.x == 0)
    for (int a = 0; a < 4; a++) partial[blockIdx.x * 4 + a] = v[a];
}

// Charge density of electrons (-w) and partners (+w) on the integer lattice.
template <typename R, int DIM, int ORDER>
__global__ __launch_bounds__(256) void k_rho(PSoA<R> S, LatticeP L, Drift<R> D, Geo g,
                                             const int* counts, double inv_dV, double* rho) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= counts[0]) return;
  int id = S.id[p];
  if (id < 0) return;
  R xi[3] = {S.xi[0][p], S.xi[1][p], S.xi[2] ? S.xi[2][p] : (R)0};
  double w = S.w[p] * inv_dV;
  Birth b = decode_id(L, id);
  Pos<R> pi = ion_pos<R, DIM>(L, id, b, D);
  Pos<R> pe = add_xi<R, DIM>(pi, xi);
  for (int sp = 0; sp < 2; sp++) {
    const Pos<R>& q = sp == 0 ? pe : pi;
    double qw = sp == 0 ? -w : w;
    R wz[ORDER + 1], wx[ORDER + 1], wy[ORDER + 1] = {};
    int bz = shape<R, ORDER>(q.c[0], q.o[0], 0, wz);
    int bx = shape<R, ORDER>(q.c[1], q.o[1], 0, wx);
    int by = 0;
    if (DIM == 3) by = shape<R, ORDER>(q.c[2], q.o[2], 0, wy);
    for (int a = 0; a <= ORDER; a++)
      for (int c = 0; c <= ORDER; c++) {
        if (DIM == 2) {
          int64_t n = gidx(g, bz + a, bx + c, 0);
          if (n >= 0) atomicAdd(&rho[n], qw * (double)wz[a] * (double)wx[c]);
        } else {
          for (int e = 0; e <= ORDER; e++) {
            int64_t n = gidx(g, bz + a, bx + c, by + e);
            if (n >= 0) atomicAdd(&rho[n], qw * (double)wz[a] * (double)wx[c] * (double)wy[e]);
          }
        }
      }
  }
}

struct GridSrc {
  const double* a;
  Geo g;
  __device__ __forceinline__ double operator()(int i, int j, int k) const {
    int64_t n = gidx(g, i, j, k);
    return n < 0 ? 0.0 : a[n];
  }
};

template <int DIM, int FZ, int FX, int FY>
__global__ __launch_bounds__(256) void k_filter_grid(Geo g, FiltK fk, const double* in,
                                                     double* out, int nbz, int nbx, int nby) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  int b = blockIdx.x;
  int by = b % nby, bx = (b / nby) % nbx, bz = b / (nby * nbx);
  GridSrc src{in, g};
  filter_tile<double, DIM, FZ, FX, FY>(g, fk, 0, bz * FZ, bx * FX, by * FY, src, out, lds);
}

// Max |div_h E - F rho| over rows [lo, hi] (partial max per block).
template <typename R, int DIM>
__global__ __launch_bounds__(kDiagBlock) void k_gauss(Geo g, Fields<R> F, const double* frho,
                                                       double idz, double idx, double idy,
                                                       int lo, int hi, double* partial) {
  __shared__ double sh[kDiagBlock];
  double m = 0.0;
  int64_t total = (int64_t)(hi - lo + 1) * g.plane;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    int i = lo + (int)(q / g.plane);
    int rem = (int)(q % g.plane);
    int j = rem / g.ny, k = rem - j * g.ny;
    int64_t n = gidx(g, i, j, k);
    double dv = ((double)F.F[2][n] - (double)at(g, F.F[2], i - 1, j, k)) * idz +
                ((double)F.F[0][n] - (double)at(g, F.F[0], i, j - 1, k)) * idx;
    if (DIM == 3) dv += ((double)F.F[1][n] - (double)at(g, F.F[1], i, j, k - 1)) * idy;
    double r = fabs(dv - frho[n]);
    if (r > m) m = r;
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = kDiagBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && sh[threadIdx.x + s] > sh[threadIdx.x])
      sh[threadIdx.x] = sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// Final reduction into out[0..]: ue, ub, ukin, ukin_drift, charge, live,
// gauss, wake_amp; lineout copied along the way.
template <typename R>
__global__ __launch_bounds__(kDiagBlock) void k_diag_final(Geo g, const R* Ez, const double* pf,
                                                            int nbf, const double* pp, int nbp,
                                                            const double* pg, int nbg,
                                                            double* out, double* lineout) {
  __shared__ double sh[6 * kDiagBlock];
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nbf; b += blockDim.x) {
    v[0] += pf[b * 2];
    v[1] += pf[b * 2 + 1];
  }
  for (int b = threadIdx.x; b < nbp; b += blockDim.x)
    for (int a = 0; a < 4; a++) v[2 + a] += pp[b * 4 + a];
  block_sum<6>(v, sh);
  double gm = 0.0, wa = 0.0;
  for (int b = threadIdx.x; b < nbg; b += blockDim.x) gm = fmax(gm, pg[b]);
  int ja = g.nx / 2, ka = g.ny / 2;
  for (int i = threadIdx.x; i < g.nz; i += blockDim.x) {
    double e = (double)Ez[gidx(g, i, ja, ka)];
    if (lineout) lineout[i] = e;
    wa = fmax(wa, fabs(e));
  }
  sh[threadIdx.x] = gm;
  sh[kDiagBlock + threadIdx.x] = wa;
  __syncthreads();
  for (int s = kDiagBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
      sh[kDiagBlock + threadIdx.x] = fmax(sh[kDiagBlock + threadIdx.x], sh[kDiagBlock + threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int a = 0; a < 6; a++) out[a] = v[a];
    out[6] = sh[0];
    out[7] = sh[kDiagBlock];
  }
}

}  // namespace bfpic
