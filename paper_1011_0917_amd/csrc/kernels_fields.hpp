// kernels_fields.hpp -- current fold + binomial filter, Yee update with Mur
// boundaries, window shift, boosted laser initialisation, field copies.
#pragma once

#include "device_common.hpp"
#include "kernels_particles.hpp"

namespace bfpic {

// Component staggering along z: 1 for half-integer rows.
// Order of the six E/B components: Ex Ey Ez Bx By Bz; currents Jx Jy Jz.
__device__ __forceinline__ int half_z_eb(int c) { return c == 2 || c == 3 || c == 4; }
__device__ __forceinline__ int half_z_j(int c) { return c == 2; }

// --------------------------------------------------------------------------
// Fold: the unfiltered current at a grid node is the sum of the LDS regions of
// every tile that covers the node, plus the overflow of the global path.
// --------------------------------------------------------------------------
template <typename R>
struct FoldK {
  const R* scratch;  // [tile][3][LV]
  int ntz, ntx, nty, ntiles;
  int gz0, gx0, gy0;  // region origin of tile (0,0,0) in grid cells
  int TZ, TX, TY, LZ, LX, LY, LV;
  Ovf<R> o;
};

template <typename R, int DIM>
__device__ __forceinline__ R fold_at(const FoldK<R>& K, const Geo& g, int comp, int i, int j,
                                     int k) {
  R acc = (R)0;
  if (g.periodic_z) i = wrapi(i, g.nz);  // halo rows of the filter may lie beyond the seam
  if (K.ntiles > 0) {
    int qz = i - K.gz0;
    if (g.periodic_z) qz = wrapi(qz, g.nz);
    int qx = wrapi(j - K.gx0, g.nx);
    int qy = DIM == 3 ? wrapi(k - K.gy0, g.ny) : 0;
    int hz = qz >= 0 ? qz / K.TZ : -((-qz + K.TZ - 1) / K.TZ);
    int hx = qx / K.TX, hy = DIM == 3 ? qy / K.TY : 0;
    const int dzmax = (K.LZ - 1) / K.TZ, dxmax = (K.LX - 1) / K.TX;
    const int dymax = DIM == 3 ? (K.LY - 1) / K.TY : 0;
    for (int dz_ = 0; dz_ <= dzmax; dz_++) {
      int tz = hz - dz_;
      int rz = qz - tz * K.TZ;
      if (g.periodic_z) {
        tz = wrapi(tz, K.ntz);
        rz = wrapi(i - (K.gz0 + tz * K.TZ), g.nz);
      }
      if (tz < 0 || tz >= K.ntz || rz < 0 || rz >= K.LZ) continue;
      for (int dx_ = 0; dx_ <= dxmax; dx_++) {
        int tx = wrapi(hx - dx_, K.ntx);
        int rx = wrapi(j - (K.gx0 + tx * K.TX), g.nx);
        if (rx >= K.LX) continue;
        for (int dy_ = 0; dy_ <= dymax; dy_++) {
          int ty = 0, ry = 0;
          if (DIM == 3) {
            ty = wrapi(hy - dy_, K.nty);
            ry = wrapi(k - (K.gy0 + ty * K.TY), g.ny);
            if (ry >= K.LY) continue;
          }
          int t = (tz * K.ntx + tx) * K.nty + ty;
          acc += K.scratch[((int64_t)t * 3 + comp) * K.LV + (rz * K.LX + rx) * K.LY + ry];
        }
      }
    }
  }
  int r0 = K.o.rows[0], r1 = K.o.rows[1];
  if (i >= r0 && i <= r1) {
    int64_t n = gidx(g, i, j, k);
    if (n >= 0) acc += K.o.J[comp][n];
  }
  return acc;
}

// Filter: per axis N passes of (1/4, 1/2, 1/4) then (-N/4, 1 + N/2, -N/4)
// when compensating; outside an open z domain the current counts as zero.
// One workgroup filters an FZ x FX [x FY] output tile of one component with
// a halo of H = N (+1) nodes, all passes in LDS.
struct FiltK {
  int passes, comp;  // N and the compensation flag
  int H;
  float a_c, b_c;    // compensation weights
};

template <typename R, int DIM, int FZ, int FX, int FY, class Src>
__device__ void filter_tile(const Geo& g, const FiltK& fk, int half_z, int i0, int j0, int k0,
                            const Src& src, R* out, R* lds) {
  const int H = fk.H;
  const int NZ = FZ + 2 * H, NX = FX + 2 * H, NY = DIM == 3 ? FY + 2 * H : 1;
  const int NV = NZ * NX * NY;
  R* A = lds;
  R* Bq = lds + NV;
  for (int v = threadIdx.x; v < NV; v += blockDim.x) {
    int r = v / (NX * NY), rem = v - r * (NX * NY);
    int s = rem / NY, u = rem - s * NY;
    int i = i0 - H + r, j = j0 - H + s, k = DIM == 3 ? k0 - H + u : 0;
    bool ok = g.periodic_z || in_domain(g, half_z, i);
    A[v] = ok ? src(i, j, k) : (R)0;
  }
  __syncthreads();
  const int naxes = DIM == 3 ? 3 : 2;
  for (int axis = 0; axis < naxes; axis++) {
    const int npass = fk.passes + (fk.comp && fk.passes > 0 ? 1 : 0);
    const int stride = axis == 0 ? NX * NY : (axis == 1 ? NY : 1);
    for (int p = 0; p < npass; p++) {
      R a = p < fk.passes ? (R)0.25 : (R)fk.a_c;
      R b = p < fk.passes ? (R)0.5 : (R)fk.b_c;
      for (int v = threadIdx.x; v < NV; v += blockDim.x) {
        int r = v / (NX * NY), rem = v - r * (NX * NY);
        int s = rem / NY, u = rem - s * NY;
        int pos = axis == 0 ? r : (axis == 1 ? s : u);
        int len = axis == 0 ? NZ : (axis == 1 ? NX : NY);
        R val;
        if (pos == 0 || pos == len - 1) val = A[v];
        else val = a * A[v - stride] + b * A[v] + a * A[v + stride];
        if (axis == 0 && !g.periodic_z && !in_domain(g, half_z, i0 - H + r)) val = (R)0;
        Bq[v] = val;
      }
      __syncthreads();
      R* t = A;
      A = Bq;
      Bq = t;
    }
  }
  for (int v = threadIdx.x; v < FZ * FX * (DIM == 3 ? FY : 1); v += blockDim.x) {
    int fy = DIM == 3 ? FY : 1;
    int r = v / (FX * fy), rem = v - r * (FX * fy);
    int s = rem / fy, u = rem - s * fy;
    int i = i0 + r, j = j0 + s, k = DIM == 3 ? k0 + u : 0;
    if (!in_domain(g, half_z, i) || j >= g.nx || (DIM == 3 && k >= g.ny)) continue;
    out[gidx(g, i, j, k)] = A[((r + H) * NX + (s + H)) * NY + (DIM == 3 ? u + H : 0)];
  }
  __syncthreads();
}

template <typename R, int DIM>
struct FoldSrc {
  const FoldK<R>* K;
  Geo g;
  int comp;
  __device__ __forceinline__ R operator()(int i, int j, int k) const {
    return fold_at<R, DIM>(*K, g, comp, i, j, k);
  }
};

template <typename R, int DIM, int FZ, int FX, int FY>
__global__ __launch_bounds__(256) void k_fold_filter(Geo g, FoldK<R> K, FiltK fk, Fields<R> Jf,
                                                     int nbz, int nbx, int nby) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* lds = reinterpret_cast<R*>(smem_raw);
  int nb = nbz * nbx * nby;
  int b = xcd_remap(blockIdx.x, nb);
  int by = b % nby, bx = (b / nby) % nbx, bz = b / (nby * nbx);
  int i0 = bz * FZ, j0 = bx * FX, k0 = by * FY;
  for (int comp = 0; comp < 3; comp++) {
    FoldSrc<R, DIM> src{&K, g, comp};
    filter_tile<R, DIM, FZ, FX, FY>(g, fk, half_z_j(comp), i0, j0, k0, src, Jf.F[comp], lds);
  }
}

// Clear the overflow rows that the global path touched this step.
template <typename R>
__global__ __launch_bounds__(256) void k_ovf_clear(Geo g, Ovf<R> o) {
  int r0 = o.rows[0], r1 = o.rows[1];
  if (r1 < r0) return;
  if (r0 < -kGuard) r0 = -kGuard;
  if (r1 > g.nz + kGuard) r1 = g.nz + kGuard;
  int64_t n = (int64_t)(r1 - r0 + 1) * g.plane;
  int64_t base = (int64_t)(r0 + kGuard) * g.plane;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    o.J[0][base + v] = (R)0;
    o.J[1][base + v] = (R)0;
    o.J[2][base + v] = (R)0;
  }
}

__global__ void k_ovf_reset(int* rows) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    rows[0] = 0x7fffffff;
    rows[1] = -0x7fffffff;
  }
}

// --------------------------------------------------------------------------
// Yee (1966) on the staggered grid with B at integer times through two half
// steps: B -= h curl E; E += dt (curl B - J); B -= h curl E.
// --------------------------------------------------------------------------
template <typename R>
struct YeeK {
  R* E[3];
  R* B[3];
  const R* J[3];
  R idz, idx, idy;  // 1/d
  R h;              // step of this update
  R mur;            // (dt - dz) / (dt + dz)
  R* save;          // [2 rows][2 comps][plane] old Ex, Ey at rows 1 and nz-1
};

template <typename R>
__device__ __forceinline__ R at(const Geo& g, const R* A, int i, int j, int k) {
  int64_t n = gidx(g, i, j, k);
  return n < 0 ? (R)0 : A[n];
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_yee_b(Geo g, YeeK<R> Y) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int nrow = g.periodic_z ? g.nz : g.nz + 1;
  if (v >= (int64_t)nrow * g.plane) return;
  int i = (int)(v / g.plane);
  int rem = (int)(v - (int64_t)i * g.plane);
  int j = rem / g.ny, k = rem - j * g.ny;
  int64_t n = gidx(g, i, j, k);
  const R* Ex = Y.E[0];
  const R* Ey = Y.E[1];
  const R* Ez = Y.E[2];
  R ey = Ey[n];
  if (i <= row_hi(g, 1)) {
    R dEz_dy = DIM == 3 ? (at(g, Ez, i, j, k + 1) - Ez[n]) * Y.idy : (R)0;
    Y.B[0][n] += Y.h * ((at(g, Ey, i + 1, j, k) - ey) * Y.idz - dEz_dy);
    Y.B[1][n] += Y.h * ((at(g, Ez, i, j + 1, k) - Ez[n]) * Y.idx -
                        (at(g, Ex, i + 1, j, k) - Ex[n]) * Y.idz);
  }
  R dEx_dy = DIM == 3 ? (at(g, Ex, i, j, k + 1) - Ex[n]) * Y.idy : (R)0;
  Y.B[2][n] += Y.h * (dEx_dy - (at(g, Ey, i, j + 1, k) - ey) * Y.idx);
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_yee_e(Geo g, YeeK<R> Y) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int nrow = g.periodic_z ? g.nz : g.nz + 1;
  if (v >= (int64_t)nrow * g.plane) return;
  int i = (int)(v / g.plane);
  int rem = (int)(v - (int64_t)i * g.plane);
  int j = rem / g.ny, k = rem - j * g.ny;
  int64_t n = gidx(g, i, j, k);
  const R* Bx = Y.B[0];
  const R* By = Y.B[1];
  const R* Bz = Y.B[2];
  bool open = !g.periodic_z;
  if (i <= row_hi(g, 1)) {
    R dBx_dy = DIM == 3 ? (Bx[n] - at(g, Bx, i, j, k - 1)) * Y.idy : (R)0;
    Y.E[2][n] += Y.h * ((By[n] - at(g, By, i, j - 1, k)) * Y.idx - dBx_dy - Y.J[2][n]);
  }
  if (open && (i == 0 || i == g.nz)) return;  // Mur planes
  if (open && (i == 1 || i == g.nz - 1)) {
    int r = i == 1 ? 0 : 1;
    int64_t q = (int64_t)rem;
    Y.save[(r * 2 + 0) * g.plane + q] = Y.E[0][n];
    Y.save[(r * 2 + 1) * g.plane + q] = Y.E[1][n];
  }
  R dBz_dy = DIM == 3 ? (Bz[n] - at(g, Bz, i, j, k - 1)) * Y.idy : (R)0;
  Y.E[0][n] += Y.h * (dBz_dy - (By[n] - at(g, By, i - 1, j, k)) * Y.idz - Y.J[0][n]);
  Y.E[1][n] += Y.h * ((Bx[n] - at(g, Bx, i - 1, j, k)) * Y.idz -
                      (Bz[n] - at(g, Bz, i, j - 1, k)) * Y.idx - Y.J[1][n]);
}

// First-order Mur at normal incidence: E0' = E1 + m (E1' - E0) at both z ends.
template <typename R>
__global__ __launch_bounds__(256) void k_mur(Geo g, YeeK<R> Y) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.plane) return;
  int j = (int)(q / g.ny), k = (int)(q - (int64_t)j * g.ny);
  for (int c = 0; c < 2; c++) {
    R* E = Y.E[c];
    int64_t n0 = gidx(g, 0, j, k), n1 = gidx(g, 1, j, k);
    int64_t m0 = gidx(g, g.nz, j, k), m1 = gidx(g, g.nz - 1, j, k);
    R old1 = Y.save[(0 * 2 + c) * g.plane + q];
    R oldm = Y.save[(1 * 2 + c) * g.plane + q];
    E[n0] = old1 + Y.mur * (E[n1] - E[n0]);
    E[m0] = oldm + Y.mur * (E[m1] - E[m0]);
  }
}

// --------------------------------------------------------------------------
// Window shift: row i takes row i + n; rows from beyond storage or outside
// the component's domain are zero.
// --------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_shift(Geo g, const R* src, R* dst, int n, int half_z) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.rows * g.plane) return;
  int row = (int)(v / g.plane);
  int64_t q = v - (int64_t)row * g.plane;
  int i = row - kGuard;
  int si = i + n;
  R val = (R)0;
  if (in_domain(g, half_z, i) && si >= -kGuard && si <= g.nz + kGuard)
    val = src[(int64_t)(si + kGuard) * g.plane + q];
  dst[v] = val;
}

// --------------------------------------------------------------------------
// Laser.  Lab vector potential A_y = a0 G(xi) Im[U e^{i(xi + phase)}] of a
// paraxial Gaussian pulse (2 i dU/dzeta + lap_perp U = 0, q = zeta - i zR),
// evaluated on the calculation frame's t' = 0 hyperplane: lab (t, z) =
// (gamma beta z', gamma z'), so xi = gamma (1 - beta) z' - z_center and
// zeta = gamma z' - z_focus.  A_y is invariant under the boost along z;
// Ey' = -dA/dt' = gamma (1 - beta) dA/dxi - gamma beta dA/dzeta.
// --------------------------------------------------------------------------
struct Cx {
  double re, im;
};
__device__ __forceinline__ Cx cmul(Cx a, Cx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ Cx cdiv(Cx a, Cx b) {
  double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ __forceinline__ Cx cexpi(Cx a) {
  double m = exp(a.re);
  return {m * cos(a.im), m * sin(a.im)};
}
__device__ __forceinline__ Cx csqrt_p(Cx a) {  // principal branch
  double r = sqrt(sqrt(a.re * a.re + a.im * a.im));
  double th = 0.5 * atan2(a.im, a.re);
  return {r * cos(th), r * sin(th)};
}

struct LaserK {
  double a0, w0, L, zc, zf, phase;
  int collimated, iz, ix, iy, dim;
  double gomb, gbeta;  // gamma (1 - beta), gamma beta
  double gamma_b;
  double Lz, Lx, Ly, xa, ya, dz, dx, dy;
};

__device__ void lab_potential(const LaserK& K, double xi, double zeta, double x, double y,
                              double& A, double& dxi, double& dzeta) {
  double G = 1.0, Gp = 0.0;
  if (K.L > 0.0) {
    if (fabs(xi) > 4.0 * K.L) {
      A = dxi = dzeta = 0.0;
      return;
    }
    double l2 = K.L * K.L;
    G = exp(-xi * xi / l2);
    Gp = -2.0 * xi / l2 * G;
  }
  Cx U = {1.0, 0.0}, dU = {0.0, 0.0};
  double r2 = K.dim == 3 ? x * x + y * y : x * x;
  if (K.w0 > 0.0) {
    if (K.collimated) {
      U = {exp(-r2 / (K.w0 * K.w0)), 0.0};
    } else {
      double zR = 0.5 * K.w0 * K.w0;
      Cx q = {zeta, -zR}, q0 = {0.0, -zR};
      Cx iq = cdiv({1.0, 0.0}, q);
      Cx ex = cexpi(cmul({0.0, 0.5 * r2}, iq));            // exp(i r^2 / (2 q))
      Cx corr = cmul({0.0, -0.5 * r2}, cmul(iq, iq));       // -i r^2 / (2 q^2)
      if (K.dim == 2) {
        U = cmul(csqrt_p(cdiv(q0, q)), ex);
        dU = cmul(U, {-0.5 * iq.re + corr.re, -0.5 * iq.im + corr.im});
      } else {
        U = cmul(cdiv(q0, q), ex);
        dU = cmul(U, {-iq.re + corr.re, -iq.im + corr.im});
      }
    }
  }
  Cx ph = {cos(xi + K.phase), sin(xi + K.phase)};
  Cx Uph = cmul(U, ph), dUph = cmul(dU, ph);
  A = K.a0 * G * Uph.im;
  dxi = K.a0 * (Gp * Uph.im + G * Uph.re);
  dzeta = K.a0 * G * dUph.im;
}

// Ey' and A' at every Ey node (i, j, k) -> (z' = i dz, x = j dx, y = (k+1/2) dy).
template <typename R>
__global__ __launch_bounds__(256) void k_laser_a(Geo g, LaserK K, R* Ey, double* A64,
                                                 double* Ey64) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int nrow = row_hi(g, 0) + 1;
  if (v >= (int64_t)nrow * g.plane) return;
  int i = (int)(v / g.plane);
  int rem = (int)(v - (int64_t)i * g.plane);
  int j = rem / g.ny, k = rem - j * g.ny;
  double zp = (double)i * K.dz;
  double x = (double)j * K.dx - K.xa;
  double y = K.dim == 3 ? ((double)k + 0.5) * K.dy - K.ya : 0.0;
  double As = 0.0, Es = 0.0;
  int my = K.dim == 3 ? K.iy : 0;
  for (int mz = -K.iz; mz <= K.iz; mz++)
    for (int mx = -K.ix; mx <= K.ix; mx++)
      for (int mm = -my; mm <= my; mm++) {
        double zz = zp + mz * K.Lz;
        double xi = K.gomb * zz - K.zc;
        double zeta = K.gamma_b * zz - K.zf;
        double a, dxi, dze;
        lab_potential(K, xi, zeta, x + mx * K.Lx, y + mm * K.Ly, a, dxi, dze);
        As += a;
        Es += K.gomb * dxi - K.gbeta * dze;
      }
  int64_t n = gidx(g, i, j, k);
  A64[n] = As;
  Ey64[n] = Es;
  Ey[n] += (R)Es;
}

// B' = curl_h (0, A', 0): Bx = -dA/dz at (i+1/2, j[, k+1/2]), Bz = dA/dx at (i, j+1/2[, k+1/2]).
template <typename R>
__global__ __launch_bounds__(256) void k_laser_b(Geo g, const double* A64, double dz, double dx,
                                                 R* Bx, R* Bz) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int nrow = row_hi(g, 0) + 1;
  if (v >= (int64_t)nrow * g.plane) return;
  int i = (int)(v / g.plane);
  int rem = (int)(v - (int64_t)i * g.plane);
  int j = rem / g.ny, k = rem - j * g.ny;
  int64_t n = gidx(g, i, j, k);
  if (i <= row_hi(g, 1)) {
    int64_t n1 = gidx(g, i + 1, j, k);
    double a1 = n1 < 0 ? 0.0 : A64[n1];
    Bx[n] += (R)(-(a1 - A64[n]) / dz);
  }
  Bz[n] += (R)((A64[gidx(g, i, j + 1, k)] - A64[n]) / dx);
}

// 3D: Ez' from discrete div E' = 0, integrated along z from the low end.
template <typename R>
__global__ __launch_bounds__(256) void k_laser_ez(Geo g, const double* Ey64, double dz, double dy,
                                                  R* Ez) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.plane) return;
  int j = (int)(q / g.ny), k = (int)(q - (int64_t)j * g.ny);
  double acc = 0.0;
  for (int i = 0; i <= row_hi(g, 1); i++) {
    acc -= dz * (Ey64[gidx(g, i, j, k)] - Ey64[gidx(g, i, j, k - 1)]) / dy;
    int64_t n = gidx(g, i, j, k);
    Ez[n] += (R)acc;
  }
}

// Field copies between the internal real type and FP64 domain arrays.
template <typename R>
__global__ __launch_bounds__(256) void k_get_field(Geo g, const R* A, double* out, int half_z) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= (int64_t)(g.nz + 1) * g.plane) return;
  int i = (int)(v / g.plane);
  double val = 0.0;
  if (in_domain(g, half_z, i)) val = (double)A[(int64_t)(i + kGuard) * g.plane + (v - (int64_t)i * g.plane)];
  out[v] = val;
}

template <typename R>
__global__ __launch_bounds__(256) void k_set_field(Geo g, R* A, const double* in, int half_z) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= (int64_t)(g.nz + 1) * g.plane) return;
  int i = (int)(v / g.plane);
  R val = in_domain(g, half_z, i) ? (R)in[v] : (R)0;
  A[(int64_t)(i + kGuard) * g.plane + (v - (int64_t)i * g.plane)] = val;
}

}  // namespace bfpic
