// kernels_witness.hpp -- witness electrons: test particles that feel the
// fields of the run and deposit no current, pushed in FP64 whatever the
// working precision, and their energy and position in the laboratory frame
// (the accelerated beam's energy gain against lab position, section
// "Modeling of up to 1 TeV stages", Fig. 4).
#pragma once

#include <math.h>

#include "device_common.hpp"
#include "kernels_particles.hpp"

namespace bfpic {

// Field fetch for the witness gather: the working-precision grid read as FP64
// (O = double, or a dual number of it).  Nodes exist on rows 0..row_hi of
// each component (open z); periodic z wraps.
template <typename R, typename O = double>
struct WideFetch {
  const R* const* F;
  Geo g;
  __device__ __forceinline__ O operator()(int comp, int i, int j, int k) const {
    const int half_z = comp == 2 || comp == 3 || comp == 4;
    if (g.periodic_z) i = wrapi(i, g.nz);
    else if (i < 0 || i > row_hi(g, half_z)) return O(0.0);
    j = wrapi(j, g.nx);
    k = g.ny > 1 ? wrapi(k, g.ny) : 0;
    return O((double)F[comp][((int64_t)(i + kGuard) * g.nx + j) * g.ny + k]);
  }
};

// Witness state, n rows of (z, x, y, u_z, u_x, u_y): position in grid cells
// relative to the window, momentum of the calculation frame.
struct WitK {
  double* s;
  int n;
  double dtd[3];  // dt / d along z, x, y
  double qdt2;    // q dt / 2, q = -1
  int galerkin;   // 1: energy-conserving gather, as the plasma's
};

struct NoSeed {
  template <typename T>
  __device__ __forceinline__ void operator()(T*, T*) const {}
};

// One step of one witness, state s updated in place: gather E, B at the
// start-of-step position with the deposit's shape, relativistic Boris
// rotation (Boris 1970) of the full momentum, move by v dt.  x and y are
// periodic; z wraps in a periodic box.  T is double, or a dual number for the
// adjoint, whose `seed` marks one gathered component as the direction.
template <typename T, int DIM, int ORDER, class Fch, class Seed>
__device__ __forceinline__ void witness_advance(const Fch& f, const Geo& g, const WitK& W, T s[6],
                                                const Seed& seed) {
  T z = s[0], x = s[1], y = s[2];
  // vectors in (x, y, z) order
  T u[3] = {s[4], s[5], s[3]};
  Pos<T> p;
  p.c[0] = (int)floor(z);
  p.o[0] = z - T((double)p.c[0]);
  p.c[1] = (int)floor(x);
  p.o[1] = x - T((double)p.c[1]);
  p.c[2] = DIM == 3 ? (int)floor(y) : 0;
  p.o[2] = DIM == 3 ? y - T((double)p.c[2]) : T(0.0);
  const int bc[3] = {p.c[0], p.c[1], p.c[2]};
  T E[3], B[3];
  gather_nodes<T, DIM, ORDER>(f, bc, p, E, B, W.galerkin != 0);
  seed(E, B);
  const T h = T(W.qdt2);
  T m[3], t[3];
#pragma unroll
  for (int a = 0; a < 3; a++) m[a] = u[a] + h * E[a];
  const T gm = sqrt(T(1.0) + m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
#pragma unroll
  for (int a = 0; a < 3; a++) t[a] = h * B[a] / gm;
  const T sf = T(2.0) / (T(1.0) + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  const T q0 = m[0] + (m[1] * t[2] - m[2] * t[1]);
  const T q1 = m[1] + (m[2] * t[0] - m[0] * t[2]);
  const T q2 = m[2] + (m[0] * t[1] - m[1] * t[0]);
  u[0] = m[0] + sf * (q1 * t[2] - q2 * t[1]) + h * E[0];
  u[1] = m[1] + sf * (q2 * t[0] - q0 * t[2]) + h * E[1];
  u[2] = m[2] + sf * (q0 * t[1] - q1 * t[0]) + h * E[2];
  const T ig = T(1.0) / sqrt(T(1.0) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  z += u[2] * ig * T(W.dtd[0]);
  if (g.periodic_z) z -= T((double)g.nz) * floor(z / T((double)g.nz));
  x += u[0] * ig * T(W.dtd[1]);
  x -= T((double)g.nx) * floor(x / T((double)g.nx));
  if (DIM == 3) {
    y += u[1] * ig * T(W.dtd[2]);
    y -= T((double)g.ny) * floor(y / T((double)g.ny));
  }
  s[0] = z;
  s[1] = x;
  s[2] = y;
  s[3] = u[2];
  s[4] = u[0];
  s[5] = u[1];
}

template <typename R, int DIM, int ORDER>
__global__ __launch_bounds__(256) void k_witness_push(Geo g, Fields<R> F, WitK W) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= W.n) return;
  double* s = W.s + (int64_t)r * 6;
  double v[6];
#pragma unroll
  for (int a = 0; a < 6; a++) v[a] = s[a];
  witness_advance<double, DIM, ORDER>(WideFetch<R>{(const R* const*)F.F, g}, g, W, v, NoSeed{});
#pragma unroll
  for (int a = 0; a < 6; a++) s[a] = v[a];
}

// The window moved forward by n cells: positions relative to it drop by n.
__global__ __launch_bounds__(256) void k_witness_shift(double* s, int n, int cells) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) s[(int64_t)r * 6] -= (double)cells;
}

// Laboratory view, rows (t, z, gamma, u_z): the witness's event (t', z') with
// z' = (z + window) dz' and its momentum boosted back from the frame moving
// at +beta_b along z: t = gb (t' + bb z'), z = gb (z' + bb t'),
// gamma = gb (gamma' + bb u'_z), u_z = gb (u'_z + bb gamma').
__global__ __launch_bounds__(256) void k_witness_lab(const double* s, int n, double tp,
                                                     double z0, double dz, double gb, double bb,
                                                     double* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double* w = s + (int64_t)r * 6;
  const double zp = z0 + w[0] * dz;
  const double uz = w[3];
  const double gp = sqrt(1.0 + uz * uz + w[4] * w[4] + w[5] * w[5]);
  double* o = out + (int64_t)r * 4;
  o[0] = gb * (tp + bb * zp);
  o[1] = gb * (zp + bb * tp);
  o[2] = gb * (gp + bb * uz);
  o[3] = gb * (uz + bb * gp);
}

}  // namespace bfpic
