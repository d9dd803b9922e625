// kernels_adjoint.hpp -- reverse sweep of the 2D PIC step, for the gradient
// of a field loss with respect to the laser amplitude and the plasma density
// profile.
//
// The step is the composition
//   gather -> push -> move -> deposit -> filter -> Yee (B half, E + Mur, B half)
// and its adjoint runs the transposes in reverse order:
//   * Yee and Mur are linear; their transposes are written out term by term
//     from the forward updates (k_adj_yee_b, k_adj_yee_e, k_adj_mur_*);
//   * the binomial filter with its open-boundary masking is symmetric, so its
//     transpose is the filter itself, applied to the current adjoint;
//   * per particle, the vector-Jacobian product of gather, push, move and
//     deposit is formed with forward-mode dual numbers: the same templated
//     step the forward kernels run is evaluated once per input direction
//     (positions 2, momenta 3, weight 1, gathered E and B 6) and contracted
//     with the adjoints of its outputs; the gathered-field directions are then
//     scattered to the field adjoint with the gather's own weights.
#pragma once

#include <type_traits>

#include "device_common.hpp"
#include "kernels_fields.hpp"
#include "kernels_particles.hpp"
#include "kernels_witness.hpp"

namespace bfpic {

// --------------------------------------------------------------------------
// Forward-mode dual number: value v and one tangent d.  Comparisons order by
// value; equality also compares the tangent, so that a branch that skips a
// zero value (an out-of-plane current with v_y = 0) still runs when the value
// has a non-zero derivative.  The math functions are hidden friends, found
// only through argument-dependent lookup.
// --------------------------------------------------------------------------
template <typename T>
struct Dual {
  T v, d;
  __device__ __forceinline__ Dual() : v((T)0), d((T)0) {}
  __device__ __forceinline__ Dual(double x) : v((T)x), d((T)0) {}
  __device__ __forceinline__ static Dual mk(T v, T d) {
    Dual r;
    r.v = v;
    r.d = d;
    return r;
  }
  __device__ __forceinline__ explicit operator int() const { return (int)v; }

  friend __device__ __forceinline__ Dual operator+(Dual a, Dual b) { return mk(a.v + b.v, a.d + b.d); }
  friend __device__ __forceinline__ Dual operator-(Dual a, Dual b) { return mk(a.v - b.v, a.d - b.d); }
  friend __device__ __forceinline__ Dual operator-(Dual a) { return mk(-a.v, -a.d); }
  friend __device__ __forceinline__ Dual operator*(Dual a, Dual b) {
    return mk(a.v * b.v, a.d * b.v + a.v * b.d);
  }
  friend __device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    const T q = a.v / b.v;
    return mk(q, (a.d - q * b.d) / b.v);
  }
  __device__ __forceinline__ Dual& operator+=(Dual b) { return *this = *this + b; }
  __device__ __forceinline__ Dual& operator-=(Dual b) { return *this = *this - b; }
  __device__ __forceinline__ Dual& operator*=(Dual b) { return *this = *this * b; }
  __device__ __forceinline__ Dual& operator/=(Dual b) { return *this = *this / b; }
  friend __device__ __forceinline__ bool operator<(Dual a, Dual b) { return a.v < b.v; }
  friend __device__ __forceinline__ bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
  friend __device__ __forceinline__ bool operator>(Dual a, Dual b) { return a.v > b.v; }
  friend __device__ __forceinline__ bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
  friend __device__ __forceinline__ bool operator==(Dual a, Dual b) { return a.v == b.v && a.d == b.d; }
  friend __device__ __forceinline__ bool operator!=(Dual a, Dual b) { return !(a == b); }
  friend __device__ __forceinline__ Dual floor(Dual a) { return mk(floor(a.v), (T)0); }
  friend __device__ __forceinline__ Dual sqrt(Dual a) {
    const T s = sqrt(a.v);
    return mk(s, s > (T)0 ? a.d / (s + s) : (T)0);
  }
  friend __device__ __forceinline__ Dual root(Dual a) {
    const T s = root(a.v);
    return mk(s, s > (T)0 ? a.d / (s + s) : (T)0);
  }
  friend __device__ __forceinline__ Dual rcp(Dual a) {
    const T r = rcp(a.v);
    return mk(r, -a.d * r * r);
  }
};

// --------------------------------------------------------------------------
// Forward-mode dual number with N tangents: one evaluation carries the
// derivatives along N input directions at once, each tangent by the rules of
// Dual.  Equality compares every tangent.
// --------------------------------------------------------------------------
template <typename T, int N>
struct DualN {
  T v, d[N];
  __device__ __forceinline__ DualN() : v((T)0) {
#pragma unroll
    for (int k = 0; k < N; k++) d[k] = (T)0;
  }
  __device__ __forceinline__ DualN(double x) : v((T)x) {
#pragma unroll
    for (int k = 0; k < N; k++) d[k] = (T)0;
  }
  // value x with tangent 1 along direction k (k outside [0, N): none)
  __device__ __forceinline__ static DualN seed(T x, int k) {
    DualN r;
    r.v = x;
#pragma unroll
    for (int m = 0; m < N; m++) r.d[m] = m == k ? (T)1 : (T)0;
    return r;
  }
  __device__ __forceinline__ explicit operator int() const { return (int)v; }

  friend __device__ __forceinline__ DualN operator+(DualN a, DualN b) {
    a.v += b.v;
#pragma unroll
    for (int k = 0; k < N; k++) a.d[k] += b.d[k];
    return a;
  }
  friend __device__ __forceinline__ DualN operator-(DualN a, DualN b) {
    a.v -= b.v;
#pragma unroll
    for (int k = 0; k < N; k++) a.d[k] -= b.d[k];
    return a;
  }
  friend __device__ __forceinline__ DualN operator-(DualN a) {
    a.v = -a.v;
#pragma unroll
    for (int k = 0; k < N; k++) a.d[k] = -a.d[k];
    return a;
  }
  friend __device__ __forceinline__ DualN operator*(DualN a, DualN b) {
    DualN r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < N; k++) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
  }
  friend __device__ __forceinline__ DualN operator/(DualN a, DualN b) {
    DualN r;
    r.v = a.v / b.v;
#pragma unroll
    for (int k = 0; k < N; k++) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
    return r;
  }
  __device__ __forceinline__ DualN& operator+=(DualN b) { return *this = *this + b; }
  __device__ __forceinline__ DualN& operator-=(DualN b) { return *this = *this - b; }
  __device__ __forceinline__ DualN& operator*=(DualN b) { return *this = *this * b; }
  __device__ __forceinline__ DualN& operator/=(DualN b) { return *this = *this / b; }
  friend __device__ __forceinline__ bool operator<(DualN a, DualN b) { return a.v < b.v; }
  friend __device__ __forceinline__ bool operator<=(DualN a, DualN b) { return a.v <= b.v; }
  friend __device__ __forceinline__ bool operator>(DualN a, DualN b) { return a.v > b.v; }
  friend __device__ __forceinline__ bool operator>=(DualN a, DualN b) { return a.v >= b.v; }
  friend __device__ __forceinline__ bool operator==(DualN a, DualN b) {
    bool e = a.v == b.v;
#pragma unroll
    for (int k = 0; k < N; k++) e = e && a.d[k] == b.d[k];
    return e;
  }
  friend __device__ __forceinline__ bool operator!=(DualN a, DualN b) { return !(a == b); }
  friend __device__ __forceinline__ DualN floor(DualN a) { return DualN((double)floor(a.v)); }
  friend __device__ __forceinline__ DualN sqrt(DualN a) {
    DualN r;
    r.v = sqrt(a.v);
    const T h = r.v > (T)0 ? (T)1 / (r.v + r.v) : (T)0;
#pragma unroll
    for (int k = 0; k < N; k++) r.d[k] = a.d[k] * h;
    return r;
  }
  friend __device__ __forceinline__ DualN root(DualN a) {
    DualN r;
    r.v = root(a.v);
    const T h = r.v > (T)0 ? (T)1 / (r.v + r.v) : (T)0;
#pragma unroll
    for (int k = 0; k < N; k++) r.d[k] = a.d[k] * h;
    return r;
  }
  friend __device__ __forceinline__ DualN rcp(DualN a) {
    DualN r;
    r.v = rcp(a.v);
    const T m = -r.v * r.v;
#pragma unroll
    for (int k = 0; k < N; k++) r.d[k] = a.d[k] * m;
    return r;
  }
};

// The step constants as constants of a dual type D (zero tangents).
template <class D, typename T>
__device__ __forceinline__ PushC<D> to_dual(const PushC<T>& p) {
  PushC<D> q;
  q.ub = p.ub;
  q.gb = p.gb;
  q.gb2 = p.gb2;
  q.qdt2 = p.qdt2;
  return q;
}

template <class D, typename T>
__device__ __forceinline__ Drift<D> to_dual(const Drift<T>& p) {
  Drift<D> q;
  q.Dint = p.Dint;
  q.Dfrac = p.Dfrac;
  return q;
}

template <class D, typename T>
__device__ __forceinline__ StepK<D> to_dual(const StepK<T>& p) {
  StepK<D> q;
  q.g = p.g;
  q.L = p.L;
  q.push = to_dual<D>(p.push);
  q.D0 = to_dual<D>(p.D0);
  q.D1 = to_dual<D>(p.D1);
  for (int a = 0; a < 3; a++) {
    q.dtd[a] = p.dtd[a];
    q.kj[a] = p.kj[a];
  }
  q.ky2d = p.ky2d;
  q.galerkin = p.galerkin;
  q.ion_moves = p.ion_moves;
  q.remove = p.remove;
  q.lim = p.lim;
  return q;
}

template <typename T>
__device__ __forceinline__ StepK<Dual<T>> dualize(const StepK<T>& p) {
  return to_dual<Dual<T>>(p);
}

// Field fetch of constant grid values as duals.
template <typename T>
struct DualFetch {
  const T* const* F;
  Geo g;
  __device__ __forceinline__ Dual<T> operator()(int comp, int i, int j, int k) const {
    // branchless: a node outside storage reads element 0 and takes zero
    const int64_t n = gidx(g, i, j, k);
    const T v = F[comp][n < 0 ? 0 : n];
    return Dual<T>(n < 0 ? 0.0 : (double)v);
  }
};

template <typename T>
struct LoadsFirst<DualFetch<T>> : std::true_type {};

// Current "sink" of the adjoint: contracts each current contribution's
// tangent with the current adjoint at its node.
template <typename T>
struct AdjJSink {
  const T* const* lj;  // adjoint of the unfiltered current, Jx Jy Jz
  Geo g;
  T* acc;
  T* accv;             // if set: the same contraction with the current's value
  __device__ __forceinline__ void add(int comp, int i, int j, int k, Dual<T> v) const {
    const int64_t n = gidx(g, i, j, k);
    const T ln = lj[comp][n < 0 ? 0 : n];  // branchless, as in DualFetch
    const T l = n < 0 ? (T)0 : ln;
    *acc += l * v.d;
    if (accv) *accv += l * v.v;
  }
};

// Seeds the tangent of one gathered field component (direction 6..11).
template <typename T>
struct SeedFields {
  int dir;
  __device__ __forceinline__ void operator()(Dual<T>* E, Dual<T>* B) const {
    if (dir >= 6 && dir < 9) E[dir - 6].d = (T)1;
    if (dir >= 9 && dir < 12) B[dir - 9].d = (T)1;
  }
};

// The same fetch and current sink for N-tangent duals: grid values are
// constants, and each current contribution's tangents are contracted with
// the current adjoint at its node into acc[0..N).
template <typename T, int N>
struct DualFetchN {
  const T* const* F;
  Geo g;
  __device__ __forceinline__ DualN<T, N> operator()(int comp, int i, int j, int k) const {
    const int64_t n = gidx(g, i, j, k);
    const T v = F[comp][n < 0 ? 0 : n];
    return DualN<T, N>(n < 0 ? 0.0 : (double)v);
  }
};

template <typename T, int N>
struct LoadsFirst<DualFetchN<T, N>> : std::true_type {};

template <typename T, int N>
struct AdjJSinkN {
  const T* const* lj;
  Geo g;
  T* acc;
  __device__ __forceinline__ void add(int comp, int i, int j, int k, DualN<T, N> v) const {
    const int64_t n = gidx(g, i, j, k);
    const T ln = lj[comp][n < 0 ? 0 : n];
    const T l = n < 0 ? (T)0 : ln;
#pragma unroll
    for (int m = 0; m < N; m++) acc[m] += l * v.d[m];
  }
};

// Transpose of the gather: g times the gather weight of every node, added to
// the field adjoint (same shapes and staggering as `gather`).
// Nodes outside a component's domain rows hold constant zeros, not state:
// they take no adjoint.
template <typename R, int ORDER, int DIM = 2>
__device__ __forceinline__ void scatter_node_weights(R* const* lf, const Geo& g, int comp, int bz,
                                                     const R* wz, int bx, const R* wx, int by,
                                                     const R* wy, R gv) {
  if (gv == (R)0) return;
  const int hz = half_z_eb(comp);
  constexpr int NY = DIM == 3 ? ORDER + 1 : 1;
#pragma unroll
  for (int a = 0; a <= ORDER; a++) {
    if (!g.periodic_z && !in_domain(g, hz, bz + a)) continue;
#pragma unroll
    for (int b = 0; b <= ORDER; b++)
#pragma unroll
      for (int c = 0; c < NY; c++) {
        const int64_t n = gidx(g, bz + a, bx + b, DIM == 3 ? by + c : 0);
        const R wgt = DIM == 3 ? wz[a] * wx[b] * wy[c] : wz[a] * wx[b];
        if (n >= 0) atomicAdd(&lf[comp][n], gv * wgt);
      }
  }
}

template <typename R, int ORDER, int DIM = 2>
__device__ __forceinline__ void gather_transpose(R* const* lf, const Geo& g, const Pos<R>& p,
                                                 const R gE[3], const R gB[3], bool gk) {
  R wz0[ORDER + 1], wz1[ORDER + 1], wx0[ORDER + 1], wx1[ORDER + 1];
  R wy0[ORDER + 1] = {}, wy1[ORDER + 1] = {};
  const int z0 = shape<R, ORDER>(p.c[0], p.o[0], 0, wz0);
  const int z1 = shape<R, ORDER>(p.c[0], p.o[0], 1, wz1);
  const int x0 = shape<R, ORDER>(p.c[1], p.o[1], 0, wx0);
  const int x1 = shape<R, ORDER>(p.c[1], p.o[1], 1, wx1);
  int y0 = 0, y1 = 0;
  if constexpr (DIM == 3) {
    y0 = shape<R, ORDER>(p.c[2], p.o[2], 0, wy0);
    y1 = shape<R, ORDER>(p.c[2], p.o[2], 1, wy1);
  }
  // the Galerkin form reads the half lattices with the reduced shape
  galerkin_half<R, ORDER>(gk, p.o[0], wz1);
  galerkin_half<R, ORDER>(gk, p.o[1], wx1);
  if constexpr (DIM == 3) galerkin_half<R, ORDER>(gk, p.o[2], wy1);
  // staggering (z, x, y): Ex (0,h,0) Ey (0,0,h) Ez (h,0,0) Bx (h,0,h) By (h,h,0) Bz (0,h,h);
  // in 2D the y entries drop out
  scatter_node_weights<R, ORDER, DIM>(lf, g, 0, z0, wz0, x1, wx1, y0, wy0, gE[0]);
  scatter_node_weights<R, ORDER, DIM>(lf, g, 1, z0, wz0, x0, wx0, y1, wy1, gE[1]);
  scatter_node_weights<R, ORDER, DIM>(lf, g, 2, z1, wz1, x0, wx0, y0, wy0, gE[2]);
  scatter_node_weights<R, ORDER, DIM>(lf, g, 3, z1, wz1, x0, wx0, y1, wy1, gB[0]);
  scatter_node_weights<R, ORDER, DIM>(lf, g, 4, z1, wz1, x1, wx1, y0, wy0, gB[1]);
  scatter_node_weights<R, ORDER, DIM>(lf, g, 5, z0, wz0, x1, wx1, y1, wy1, gB[2]);
}

// Per-slot adjoint state: adjoints of the displacement and momentum carried
// backwards from step to step, and the accumulated weight adjoint.
template <typename R>
struct AdjSlots {
  R* lxi[3];   // z, x (, y)
  R* ldu[3];
  double* lw;
};

// Particle state of one taped step (after that step's injection).
template <typename R>
struct TapeParticles {
  const int* id;
  const R* xi[3];     // z, x (, y)
  const R* du[3];
  const R* w;         // weights (constant per slot)
  const int* count;   // number of slots during the step
};

// One reverse particle step (2D): for every live slot, the vector-Jacobian
// product of (xi, du, w, E_p, B_p) -> (xi', du', J) with the adjoints of xi',
// du' (in A, overwritten with those of xi, du) and of J (lj); the weight
// adjoint accumulates; the E_p, B_p directions go to the field adjoint lf.
template <typename R, int ORDER>
__global__ __launch_bounds__(256) void k_adj_particles(StepK<R> P, Fields<R> F,
                                                       TapeParticles<R> T, Fields<R> LJ,
                                                       Fields<R> LF, AdjSlots<R> A) {
  using D = Dual<R>;
  const StepK<D> PD = dualize(P);
  const Geo& g = P.g;
  const int n = *T.count;
  DualFetch<R> fetch{(const R* const*)F.F, g};
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    const int id = T.id[p];
    if (id < 0) continue;
    const R xi0 = T.xi[0][p], xi1 = T.xi[1][p];
    const R du0 = T.du[0][p], du1 = T.du[1][p], du2 = T.du[2][p];
    const R w = T.w[p];
    const Birth b = decode_id(P.L, id);
    R r[3];
    birth_offsets<R, 2>(P.L, id, r);
    D rd[3] = {D((double)r[0]), D((double)r[1]), D(0.0)};
    const Pos<D> i0 = ion_at<D, 2>(b, rd, PD.D0);
    const Pos<D> i1 = ion_at<D, 2>(b, rd, PD.D1);
    const R lx0 = A.lxi[0][p], lx1 = A.lxi[1][p];
    const R lu0 = A.ldu[0][p], lu1 = A.ldu[1][p], lu2 = A.ldu[2][p];
    R gdir[12];
    // The current is linear in the weight and nothing else depends on it, so
    // the weight direction is the current's value contracted with its adjoint,
    // divided by w: taken from the first pass (a zero weight runs its own).
    R accv = (R)0;
#pragma unroll 1
    for (int dir = 0; dir < 12; dir++) {
      if (dir == 5 && w != (R)0) {
        gdir[5] = accv / w;
        continue;
      }
      D xi[3] = {D((double)xi0), D((double)xi1), D(0.0)};
      D du[3] = {D((double)du0), D((double)du1), D((double)du2)};
      D wd = D((double)w);
      if (dir < 2) xi[dir].d = (R)1;
      else if (dir < 5) du[dir - 2].d = (R)1;
      else if (dir == 5) wd.d = (R)1;
      R acc = (R)0;
      AdjJSink<R> snk{(const R* const*)LJ.F, g, &acc, dir == 0 ? &accv : nullptr};
      const Pos<D> e0 = add_xi<D, 2>(i0, xi);
      const int bc[3] = {e0.c[0], e0.c[1], 0};
      (void)particle_step<D, 2, ORDER>(PD, fetch, snk, bc, e0, i0, i1, xi, du, wd,
                                       SeedFields<R>{dir});
      gdir[dir] = acc + lx0 * xi[0].d + lx1 * xi[1].d + lu0 * du[0].d + lu1 * du[1].d +
                  lu2 * du[2].d;
    }
    A.lxi[0][p] = gdir[0];
    A.lxi[1][p] = gdir[1];
    A.ldu[0][p] = gdir[2];
    A.ldu[1][p] = gdir[3];
    A.ldu[2][p] = gdir[4];
    A.lw[p] += (double)gdir[5];
    // gather transpose at the primal position
    R xr[3] = {xi0, xi1, (R)0};
    const Pos<R> e0p = add_xi<R, 2>(ion_at<R, 2>(b, r, P.D0), xr);
    const R gE[3] = {gdir[6], gdir[7], gdir[8]}, gB[3] = {gdir[9], gdir[10], gdir[11]};
    gather_transpose<R, ORDER>(LF.F, g, e0p, gE, gB, P.galerkin != 0);
  }
}

// The same reverse particle step by stages.  The step factors as
//   (xi) -> gather -> (E, B);  (E, B, du) -> push -> (du', v);
//   xi' = xi + v dt/d;  (xi, xi', w, v_y) -> deposit -> J,
// and each stage's Jacobian has few input directions, so each is evaluated
// once on a dual type with one tangent per input of that stage: the gather
// on 2 (the displacement), the push on 9 (fields and momentum), the deposit
// on 6 (old and new displacement, weight, v_y; the deposit is contracted
// with the current adjoint at once).  The chain rule then gives the same
// vector-Jacobian product as the twelve passes of k_adj_particles, from the
// same templated gather, push and deposit.
template <typename R, int ORDER, int DIM = 2>
__global__ __launch_bounds__(256) void k_adj_particles_staged(StepK<R> P, Fields<R> F,
                                                              TapeParticles<R> T, Fields<R> LJ,
                                                              Fields<R> LF, AdjSlots<R> A) {
  // 2D: the gather on 2 tangents, the deposit on 6 (xi, xi', w, v_y: the
  // out-of-plane current); 3D: 3 and 7 (xi, xi', w)
  constexpr int ND = DIM == 3 ? 7 : 6;
  using DG = DualN<R, DIM>;
  using D9 = DualN<R, 9>;
  using DD = DualN<R, ND>;
  const StepK<DG> PG = to_dual<DG>(P);
  const PushC<D9> push9 = to_dual<D9>(P.push);
  const StepK<DD> PD = to_dual<DD>(P);
  const Geo& g = P.g;
  const int n = *T.count;
  const bool gk = P.galerkin != 0;
  DualFetchN<R, DIM> fetch{(const R* const*)F.F, g};
  // Slots stay in creation order during a taped run (no sort): whole lattice
  // columns, the ppc slots of a cell in a row.  They are taken slot-major
  // (thread q: cell q mod m, slot q / m), so that the lanes of a wave scatter
  // their field adjoints around distinct cells rather than onto one cell's
  // nodes.
  const int ppc = P.L.ppc;
  const bool il = ppc > 1 && n % ppc == 0;
  const int m = il ? n / ppc : 1;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const int qs = q / m;
    const int p = il ? (q - qs * m) * ppc + qs : q;
    const int id = T.id[p];
    if (id < 0) continue;
    const R xi[3] = {T.xi[0][p], T.xi[1][p], DIM == 3 ? T.xi[2][p] : (R)0};
    const R w = T.w[p];
    const Birth b = decode_id(P.L, id);
    R r[3];
    birth_offsets<R, DIM>(P.L, id, r);
    // gather: E, B and their derivatives along the displacement
    DG EG[3], BG[3];
    int bc[3];
    {
      const DG rg[3] = {DG((double)r[0]), DG((double)r[1]), DG((double)r[2])};
      DG xg[3];
#pragma unroll
      for (int a = 0; a < 3; a++) xg[a] = a < DIM ? DG::seed(xi[a], a) : DG(0.0);
      const Pos<DG> e0 = add_xi<DG, DIM>(ion_at<DG, DIM>(b, rg, PG.D0), xg);
      bc[0] = e0.c[0];
      bc[1] = e0.c[1];
      bc[2] = DIM == 3 ? e0.c[2] : 0;
      gather<DG, DIM, ORDER>(fetch, bc, e0, EG, BG, gk);
    }
    // push: derivatives along (E, B, du)
    D9 E9[3], B9[3], du9[3], dv9[3], gam9;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      E9[c] = D9::seed(EG[c].v, c);
      B9[c] = D9::seed(BG[c].v, 3 + c);
      du9[c] = D9::seed(T.du[c][p], 6 + c);
    }
    boris_split(push9, E9, B9, du9, dv9, gam9);
    // move, as the forward step: position axes (z, x, y) take v_z, v_x, v_y
    const R xnv[3] = {xi[0] + dv9[2].v * P.dtd[0], xi[1] + dv9[0].v * P.dtd[1],
                      DIM == 3 ? xi[2] + dv9[1].v * P.dtd[2] : (R)0};
    // deposit, contracted with the current adjoint: derivatives along
    // (xi, xi', w[, v_y])
    R s[ND];
#pragma unroll
    for (int k = 0; k < ND; k++) s[k] = (R)0;
    {
      const DD rd[3] = {DD((double)r[0]), DD((double)r[1]), DD((double)r[2])};
      const Pos<DD> i0 = ion_at<DD, DIM>(b, rd, PD.D0);
      const Pos<DD> i1 = ion_at<DD, DIM>(b, rd, PD.D1);
      DD xo[3], xn[3];
#pragma unroll
      for (int a = 0; a < 3; a++) {
        xo[a] = a < DIM ? DD::seed(xi[a], a) : DD(0.0);
        xn[a] = a < DIM ? DD::seed(xnv[a], DIM + a) : DD(0.0);
      }
      const DD wd = DD::seed(w, 2 * DIM);
      const Pos<DD> e0 = add_xi<DD, DIM>(i0, xo);
      const Pos<DD> e1 = add_xi<DD, DIM>(i1, xn);
      AdjJSinkN<R, ND> snk{(const R* const*)LJ.F, g, s};
      if constexpr (DIM == 2) {
        const DD vy = DD::seed(dv9[1].v, 5);
        bool done = false;
        if constexpr (ORDER == 1) done = deposit2d_pair<DD>(PD, snk, bc, e0, e1, i0, i1, xo, xn, wd, vy);
        if (!done) deposit2d<DD, ORDER>(PD, snk, bc, e0, e1, i0, i1, wd, vy, true);
      } else {
        deposit3d<DD, ORDER>(PD, snk, bc, e0, e1, i0, i1, wd, true);
      }
    }
    // chain rule, outputs to inputs
    R axn[3] = {(R)0, (R)0, (R)0};
#pragma unroll
    for (int a = 0; a < DIM; a++) axn[a] = A.lxi[a][p] + s[DIM + a];
    const R adv[3] = {axn[1] * P.dtd[1], DIM == 3 ? axn[2] * P.dtd[2] : s[ND - 1],
                      axn[0] * P.dtd[0]};
    const R adu[3] = {A.ldu[0][p], A.ldu[1][p], A.ldu[2][p]};
    R ain[9];
#pragma unroll
    for (int k = 0; k < 9; k++) {
      R a = (R)0;
#pragma unroll
      for (int c = 0; c < 3; c++) a += adu[c] * du9[c].d[k] + adv[c] * dv9[c].d[k];
      ain[k] = a;
    }
#pragma unroll
    for (int a = 0; a < DIM; a++) {
      R axo = s[a] + axn[a];
#pragma unroll
      for (int c = 0; c < 3; c++) axo += ain[c] * EG[c].d[a] + ain[3 + c] * BG[c].d[a];
      A.lxi[a][p] = axo;
    }
    A.ldu[0][p] = ain[6];
    A.ldu[1][p] = ain[7];
    A.ldu[2][p] = ain[8];
    A.lw[p] += (double)s[2 * DIM];
    // gather transpose at the primal position
    const R xr[3] = {xi[0], xi[1], xi[2]};
    const Pos<R> e0p = add_xi<R, DIM>(ion_at<R, DIM>(b, r, P.D0), xr);
    gather_transpose<R, ORDER, DIM>(LF.F, g, e0p, ain, ain + 3, gk);
  }
}

// --------------------------------------------------------------------------
// Transposes of the Yee updates.  The forward updates are
//   B half step (h = dt/2), rows [0, nrow):
//     Bx += h ((Ey(i+1) - Ey(i)) / dz - (Ez(k+1) - Ez(k)) / dy)   [half-z rows]
//     By += h ((Ez(j+1) - Ez(j)) / dx - (Ex(i+1) - Ex(i)) / dz)   [half-z rows]
//     Bz += h ((Ex(k+1) - Ex(k)) / dy - (Ey(j+1) - Ey(j)) / dx)
//   E step (h = dt), Ex, Ey on rows R (open z: 1..nz-1, the ends are Mur's):
//     Ez += h ((By(j) - By(j-1)) / dx - (Bx(k) - Bx(k-1)) / dy - Jz)   [half-z rows]
//     Ex += h ((Bz(k) - Bz(k-1)) / dy - (By(i) - By(i-1)) / dz - Jx)
//     Ey += h ((Bx(i) - Bx(i-1)) / dz - (Bz(j) - Bz(j-1)) / dx - Jy)
// (the y differences only in 3D).  Adjoint arrays are zero outside each
// component's domain rows, so the neighbour reads below need no row tests
// beyond R.
// --------------------------------------------------------------------------
template <typename R>
struct AdjYeeK {
  R* LE[3];
  R* LB[3];
  R* LJ[3];  // adjoint of the filtered current (written by the E transpose)
  R idz, idx, idy;
  R h;
};

// lambda_E += h K_E^T lambda_B (the B half step's transpose; lambda_B unchanged)
template <typename R, int DIM = 2>
__global__ __launch_bounds__(256) void k_adj_yee_b(Geo g, AdjYeeK<R> Y) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nrow = g.periodic_z ? g.nz : g.nz + 1;
  if (v >= (int64_t)nrow * g.plane) return;
  const int i = (int)(v / g.plane);
  const int rem = (int)(v - (int64_t)i * g.plane);
  const int j = rem / g.ny, k = rem - j * g.ny;
  const int64_t n = gidx(g, i, j, k);
  const R* LBx = Y.LB[0];
  const R* LBy = Y.LB[1];
  const R* LBz = Y.LB[2];
  const R h = Y.h;
  R ex = h * Y.idz * (LBy[n] - at(g, LBy, i - 1, j, k));
  if (DIM == 3) ex += h * Y.idy * (at(g, LBz, i, j, k - 1) - LBz[n]);
  Y.LE[0][n] += ex;
  Y.LE[1][n] += h * Y.idz * (at(g, LBx, i - 1, j, k) - LBx[n]) +
                h * Y.idx * (LBz[n] - at(g, LBz, i, j - 1, k));
  if (i <= row_hi(g, 1)) {
    R ez = h * Y.idx * (at(g, LBy, i, j - 1, k) - LBy[n]);
    if (DIM == 3) ez += h * Y.idy * (LBx[n] - at(g, LBx, i, j, k - 1));
    Y.LE[2][n] += ez;
  }
}

// lambda_B += h K_B^T lambda_E|R ; lambda_J = -h lambda_E|R (lambda_E unchanged)
template <typename R>
__device__ __forceinline__ R lam_r(const Geo& g, const R* L, int i, int j, int k) {
  // lambda_E of Ex / Ey restricted to the rows the E step updates
  if (!g.periodic_z && (i <= 0 || i >= g.nz)) return (R)0;
  return at(g, L, i, j, k);
}

template <typename R, int DIM = 2>
__global__ __launch_bounds__(256) void k_adj_yee_e(Geo g, AdjYeeK<R> Y) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nrow = g.periodic_z ? g.nz : g.nz + 1;
  if (v >= (int64_t)nrow * g.plane) return;
  const int i = (int)(v / g.plane);
  const int rem = (int)(v - (int64_t)i * g.plane);
  const int j = rem / g.ny, k = rem - j * g.ny;
  const int64_t n = gidx(g, i, j, k);
  const R* LEx = Y.LE[0];
  const R* LEy = Y.LE[1];
  const R* LEz = Y.LE[2];
  const R h = Y.h;
  if (i <= row_hi(g, 1)) {
    Y.LB[1][n] += h * Y.idx * (LEz[n] - at(g, LEz, i, j + 1, k)) +
                  h * Y.idz * (lam_r(g, LEx, i + 1, j, k) - lam_r(g, LEx, i, j, k));
    R bx = h * Y.idz * (lam_r(g, LEy, i, j, k) - lam_r(g, LEy, i + 1, j, k));
    if (DIM == 3) bx += h * Y.idy * (at(g, LEz, i, j, k + 1) - LEz[n]);
    Y.LB[0][n] += bx;
    Y.LJ[2][n] = -h * LEz[n];
  }
  R bz = h * Y.idx * (lam_r(g, LEy, i, j + 1, k) - lam_r(g, LEy, i, j, k));
  if (DIM == 3) bz += h * Y.idy * (lam_r(g, LEx, i, j, k) - lam_r(g, LEx, i, j, k + 1));
  Y.LB[2][n] += bz;
  Y.LJ[0][n] = -h * lam_r(g, LEx, i, j, k);
  Y.LJ[1][n] = -h * lam_r(g, LEy, i, j, k);
}

// Mur at both z ends, forward: E(0) <- E_old(1) + m (E_new(1) - E_old(0)), the
// same at nz from nz-1.  Transpose in two parts around the E transpose: first
// the adjoint of E_new(1) takes m lambda(0) and lambda(0) becomes -m lambda(0)
// (the adjoint of E_old(0)); after the E transpose the adjoint of E_old(1)
// takes the saved lambda(0).  One thread per node q of a z plane.
template <typename R>
__global__ __launch_bounds__(256) void k_adj_mur_pre(Geo g, AdjYeeK<R> Y, R mur, R* save) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.plane) return;
  const int64_t n0 = (int64_t)kGuard * g.plane + q, n1 = n0 + g.plane;
  const int64_t m0 = (int64_t)(g.nz + kGuard) * g.plane + q, m1 = m0 - g.plane;
  for (int c = 0; c < 2; c++) {
    R* L = Y.LE[c];
    const R t0 = L[n0], tm = L[m0];
    save[(0 * 2 + c) * g.plane + q] = t0;
    save[(1 * 2 + c) * g.plane + q] = tm;
    L[n1] += mur * t0;
    L[m1] += mur * tm;
    L[n0] = -mur * t0;
    L[m0] = -mur * tm;
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_adj_mur_post(Geo g, AdjYeeK<R> Y, const R* save) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.plane) return;
  const int64_t n1 = (int64_t)(1 + kGuard) * g.plane + q;
  const int64_t m1 = (int64_t)(g.nz - 1 + kGuard) * g.plane + q;
  for (int c = 0; c < 2; c++) {
    R* L = Y.LE[c];
    L[n1] += save[(0 * 2 + c) * g.plane + q];
    L[m1] += save[(1 * 2 + c) * g.plane + q];
  }
}

// --------------------------------------------------------------------------
// The filter on a plain grid array of the working precision (the current
// adjoint); rows outside the component's domain are not written.
// --------------------------------------------------------------------------
template <typename R>
struct GridSrcR {
  const R* a;
  Geo g;
  __device__ __forceinline__ R operator()(int i, int j, int k) const {
    const int64_t n = gidx(g, i, j, k);
    return n < 0 ? (R)0 : a[n];
  }
};

template <typename R, int FZ, int FX>
__global__ __launch_bounds__(256) void k_filter_grid_r(Geo g, FiltK fk, const R* in, R* out,
                                                       int half_z, int nbz, int nbx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* lds = reinterpret_cast<R*>(smem_raw);
  const int b = blockIdx.x;
  const int bx = b % nbx, bz = b / nbx;
  GridSrcR<R> src{in, g};
  filter_tile<R, 2, FZ, FX, 1>(g, fk, half_z, bz * FZ, bx * FX, 0, src, out, lds);
}

// The same for the three current components in one launch (blockIdx.y: Jx,
// Jy, Jz; Jz on the half rows).
template <typename R>
struct Grid3R {
  const R* in[3];
  R* out[3];
};

template <typename R, int FZ, int FX>
__global__ __launch_bounds__(256) void k_filter_grid_r3(Geo g, FiltK fk, Grid3R<R> io, int nbz,
                                                        int nbx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* lds = reinterpret_cast<R*>(smem_raw);
  const int c = blockIdx.y;
  const int b = blockIdx.x;
  const int bx = b % nbx, bz = b / nbx;
  GridSrcR<R> src{io.in[c], g};
  filter_tile<R, 2, FZ, FX, 1>(g, fk, c == 2 ? 1 : 0, bz * FZ, bx * FX, 0, src, io.out[c], lds);
}

// 3D: F x F x F output tiles (the filter's three axes in LDS).
template <typename R, int F>
__global__ __launch_bounds__(256) void k_filter_grid_r3d(Geo g, FiltK fk, Grid3R<R> io, int nbz,
                                                         int nbx, int nby) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* lds = reinterpret_cast<R*>(smem_raw);
  const int c = blockIdx.y;
  const int b = blockIdx.x;
  const int by = b % nby, bx = (b / nby) % nbx, bz = b / (nby * nbx);
  GridSrcR<R> src{io.in[c], g};
  filter_tile<R, 3, F, F, F>(g, fk, c == 2 ? 1 : 0, bz * F, bx * F, by * F, src, io.out[c], lds);
}

// --------------------------------------------------------------------------
// Transpose of the window shift.  The shift by n sets, on a component's
// domain rows i, F'(i) = F(i + n) (zero where i + n leaves storage) and
// leaves zeros elsewhere; the rows outside the domain hold no state.  So
// lambda(j) = lambda'(j - n) on domain rows j whose source row j - n is a
// domain row, else zero.  blockIdx.y: Ex Ey Ez Bx By Bz (Ez, Bx, By on the
// half rows).
// --------------------------------------------------------------------------
template <typename R>
struct ShiftAdj {
  const R* src[6];
  R* dst[6];
};

template <typename R>
__global__ __launch_bounds__(256) void k_shift_adj(Geo g, ShiftAdj<R> S, int n) {
  const int c = blockIdx.y;
  const int half = c == 2 || c == 3 || c == 4;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.rows * g.plane) return;
  const int row = (int)(v / g.plane);
  const int64_t q = v - (int64_t)row * g.plane;
  const int j = row - kGuard, i = j - n;
  R val = (R)0;
  if (in_domain(g, half, j) && in_domain(g, half, i))
    val = S.src[c][(int64_t)(i + kGuard) * g.plane + q];
  S.dst[c][v] = val;
}

// --------------------------------------------------------------------------
// Several device copies in one launch (the per-step tape): copy blockIdx.y
// moves words[y] 32-bit words; 16-byte chunks where both ends are 16-byte
// aligned, then the remaining words.
// --------------------------------------------------------------------------
constexpr int kMaxCopies = 16;
struct CopyBatch {
  const void* src[kMaxCopies];
  void* dst[kMaxCopies];
  int64_t words[kMaxCopies];
};

__global__ __launch_bounds__(256) void k_copy_batch(CopyBatch cb) {
  const int c = blockIdx.y;
  const int64_t nw = cb.words[c];
  const uint32_t* s = reinterpret_cast<const uint32_t*>(cb.src[c]);
  uint32_t* d = reinterpret_cast<uint32_t*>(cb.dst[c]);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t done = 0;
  if (((reinterpret_cast<uintptr_t>(s) | reinterpret_cast<uintptr_t>(d)) & 15) == 0) {
    const int64_t n4 = nw / 4;
    const uint4* s4 = reinterpret_cast<const uint4*>(s);
    uint4* d4 = reinterpret_cast<uint4*>(d);
    for (int64_t q = t0; q < n4; q += stride) d4[q] = s4[q];
    done = n4 * 4;
  }
  for (int64_t q = done + t0; q < nw; q += stride) d[q] = s[q];
}

// --------------------------------------------------------------------------
// Loss: the mean of Ez over a node box [i0, i1] x [j0, j1] (x [k0, k1] in 3D;
// k0 = k1 = 0 in 2D), scaled, added to acc (forward) or added to the Ez
// adjoint (reverse).
// --------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_loss_ez(Geo g, const R* Ez, int i0, int i1, int j0,
                                                 int j1, int k0, int k1, double scale,
                                                 double* acc) {
  __shared__ double sh[256];
  const int ni = i1 - i0 + 1, nj = j1 - j0 + 1, nk = k1 - k0 + 1;
  double s = 0.0;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < ni * nj * nk;
       q += gridDim.x * blockDim.x) {
    const int i = i0 + q / (nj * nk), rq = q % (nj * nk);
    const int j = j0 + rq / nk, k = k0 + rq % nk;
    s += (double)Ez[gidx(g, i, j, k)];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(acc, sh[0] * scale);
}

template <typename R>
__global__ __launch_bounds__(256) void k_loss_ez_adj(Geo g, R* LEz, int i0, int i1, int j0,
                                                     int j1, int k0, int k1, R scale) {
  const int ni = i1 - i0 + 1, nj = j1 - j0 + 1, nk = k1 - k0 + 1;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ni * nj * nk) return;
  const int rq = q % (nj * nk);
  LEz[gidx(g, i0 + q / (nj * nk), j0 + rq / nk, k0 + rq % nk)] += scale;
}

// --------------------------------------------------------------------------
// Parameter gradients.
//   a0: the initial fields are a0 times the unit pulse, so
//       dL/da0 = <lambda_F(0), F(0)> / a0   (block partial sums of the product)
//   density: w = gamma_b n_lab(z_lab) dV / ppc with n_lab piecewise linear in
//       the knot values, so dL/dn_m = sum_p lambda_w gamma_b dV/ppc phi_m(z_lab)
//       with phi_m the hat function of knot m (one value for a uniform n).
// --------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_dot_fields(const R* a, const R* b, int64_t n,
                                                    double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x)
    s += (double)a[q] * (double)b[q];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, sh[0]);
}

constexpr int kMaxKnots = 32;

__global__ __launch_bounds__(256) void k_knot_grad(const int* id_birth, const double* lw,
                                                   int64_t nslots, LatticeP L, DensityK d,
                                                   double* out /* [kMaxKnots] */) {
  __shared__ double sh[kMaxKnots];
  const int nk = d.nknots >= 2 ? d.nknots : 1;
  if ((int)threadIdx.x < kMaxKnots) sh[threadIdx.x] = 0.0;
  __syncthreads();
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nslots;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int id = id_birth[p];
    if (id < 0) continue;
    const Birth b = decode_id(L, id);
    const double c = lw[p] * d.gamma_b * d.dV_over_ppc * birth_channel(d, L, id, b);
    if (d.nknots < 2) {
      atomicAdd(&sh[0], c);
      continue;
    }
    const double rz = (double)birth_offset<double>(L, id, 0);
    const double zl = d.gamma_b * ((double)b.k + rz) * d.dz;
    if (zl < d.kz[0] || zl > d.kz[d.nknots - 1]) continue;
    for (int m = 0; m + 1 < d.nknots; m++) {
      if (zl <= d.kz[m + 1]) {
        const double f = (zl - d.kz[m]) / (d.kz[m + 1] - d.kz[m]);
        atomicAdd(&sh[m], c * (1.0 - f));
        atomicAdd(&sh[m + 1], c * f);
        break;
      }
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nk) atomicAdd(&out[threadIdx.x], sh[threadIdx.x]);
}

// Birth ids of the slots: a slot keeps the id it was created with after its
// particle is removed (the weight adjoint is needed for every particle).
__global__ __launch_bounds__(256) void k_note_ids(const int* id, const int* counts, int* id_birth) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= counts[0]) return;
  const int v = id[p];
  if (v >= 0) id_birth[p] = v;
}

// --------------------------------------------------------------------------
// Witness electrons in the adjoint.  Loss term: sc times the sum over the
// witnesses of the lab-frame energy after the last step,
// gamma_lab = gb (gamma' + bb u'_z) (sc = weight / number of witnesses).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_witness_energy(const double* s, int n, double sc,
                                                        double gb, double bb, double* acc) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double* w = s + (int64_t)r * 6;
  const double gp = sqrt(1.0 + w[3] * w[3] + w[4] * w[4] + w[5] * w[5]);
  atomicAdd(acc, sc * gb * (gp + bb * w[3]));
}

// Gradient of that term with respect to the final witness state (the
// positions take none).
__global__ __launch_bounds__(256) void k_witness_energy_seed(const double* s, int n, double sc,
                                                             double gb, double bb, double* lam) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double* w = s + (int64_t)r * 6;
  double* l = lam + (int64_t)r * 6;
  const double ig = 1.0 / sqrt(1.0 + w[3] * w[3] + w[4] * w[4] + w[5] * w[5]);
  l[0] = 0.0;
  l[1] = 0.0;
  l[2] = 0.0;
  l[3] = sc * gb * (w[3] * ig + bb);
  l[4] = sc * gb * w[4] * ig;
  l[5] = sc * gb * w[5] * ig;
}

// One reverse witness step (2D): the vector-Jacobian product of
// (state, E_p, B_p) -> state' with the adjoint of state' (lam, overwritten
// with that of state), formed with dual numbers over the 12 input
// directions; the E_p, B_p directions go to the field adjoint lf through the
// gather's transpose.  W.s holds the taped start-of-step states.
template <typename R, int ORDER, int DIM = 2>
__global__ __launch_bounds__(256) void k_adj_witness(Geo g, Fields<R> F, WitK W, double* lam,
                                                     Fields<R> LF) {
  using D = Dual<double>;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= W.n) return;
  const double* s0 = W.s + (int64_t)r * 6;
  double* l = lam + (int64_t)r * 6;
  double lo[6], gdir[12];
#pragma unroll
  for (int a = 0; a < 6; a++) lo[a] = l[a];
  const WideFetch<R, D> f{(const R* const*)F.F, g};
#pragma unroll 1
  for (int dir = 0; dir < 12; dir++) {
    D v[6];
#pragma unroll
    for (int a = 0; a < 6; a++) v[a] = D(s0[a]);
    if (dir < 6) v[dir].d = 1.0;
    witness_advance<D, DIM, ORDER>(f, g, W, v, SeedFields<double>{dir});
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 6; a++) acc += lo[a] * v[a].d;
    gdir[dir] = acc;
  }
#pragma unroll
  for (int a = 0; a < 6; a++) l[a] = gdir[a];
  Pos<R> p;
  p.c[0] = (int)floor(s0[0]);
  p.o[0] = (R)(s0[0] - (double)p.c[0]);
  p.c[1] = (int)floor(s0[1]);
  p.o[1] = (R)(s0[1] - (double)p.c[1]);
  p.c[2] = DIM == 3 ? (int)floor(s0[2]) : 0;
  p.o[2] = DIM == 3 ? (R)(s0[2] - (double)p.c[2]) : (R)0;
  const R gE[3] = {(R)gdir[6], (R)gdir[7], (R)gdir[8]};
  const R gB[3] = {(R)gdir[9], (R)gdir[10], (R)gdir[11]};
  gather_transpose<R, ORDER, DIM>(LF.F, g, p, gE, gB, W.galerkin != 0);
}

}  // namespace bfpic
