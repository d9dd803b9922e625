// kernels_particles.hpp -- gather, Boris push, move and Esirkepov deposit of
// every electron and its drifting ion partner; plasma creation and export.
//
// Particle state (structure of arrays, one slot per electron):
//   id          lattice identity; the ion partner's birth spot is derived from it
//   xi[3]       electron displacement from its partner, in cells (z, x, y)
//   du[3]       peculiar momentum u - u_b z, (x, y, z) order
//   w           weight (real particles per macro-particle)
// The partner never stores a position: it sits at its birth spot minus the
// rigid drift D of the lab-rest plasma (plus the window displacement).
#pragma once

#include <climits>
#include <type_traits>

#include "device_common.hpp"

namespace bfpic {

template <typename R>
struct PSoA {
  int* id;
  R* xi[3];
  R* du[3];
  R* w;
};

template <typename R>
struct Fields {
  R* F[6];  // Ex Ey Ez Bx By Bz
};

// Per-step constants of the particle kernels.
template <typename R>
struct StepK {
  Geo g;
  LatticeP L;
  PushC<R> push;
  Drift<R> D0, D1;   // drift at the start and end of the step
  R dtd[3];          // dt / d along z, x, y: cells moved per unit velocity
  R kj[3];           // prefix scale per unit q w: Jz 1/(dx[dy] dt), Jx 1/(dz[dy] dt), Jy 1/(dz dx dt)
  R ky2d;            // 2D out-of-plane: 1/(dz dx)
  int galerkin;      // 1: energy-conserving gather (one order lower on half nodes)
  int ion_moves;     // the partner drifts (boosted frame)
  int remove;        // open z: drop pairs beyond `lim` cells outside [0, nz]
  int lim;
};

// Overflow sink for particles outside their tile's LDS region.
template <typename R>
struct Ovf {
  R* J[3];           // Jx Jy Jz on the grid (zero between steps)
  long long* Jq[3];  // the same memory as fixed-point sums (deterministic mode)
  int* rows;         // [0] min row touched, [1] max row touched
};

// Round a value already expressed in fixed-point units to the nearest int64
// (ties to even), valid for |x| < 2^51: adding 1.5 * 2^52 leaves the rounded
// integer in the low mantissa bits of the sum.
__device__ __forceinline__ long long to_fixed(double x) {
  const double t = x + 6755399441055744.0;
  return (long long)__double_as_longlong(t) - 0x4338000000000000LL;
}

// --------------------------------------------------------------------------
// Field fetchers and current sinks.  Coordinates are node indices in the
// fetcher's own frame: LDS-relative for the tiled path, absolute (unwrapped)
// grid indices for the global path.
// --------------------------------------------------------------------------
// Offset of node (i, j, k) in an LDS region of LX x LY columns.  Region
// coordinates are small and non-negative, so the products use the full-rate
// 24-bit multiply.
template <int LX, int LY>
__device__ __forceinline__ int lds_index(int i, int j, int k) {
  const unsigned r = __umul24((unsigned)i, (unsigned)LX) + (unsigned)j;
  return (int)(LY == 1 ? r : __umul24(r, (unsigned)LY) + (unsigned)k);
}

template <typename R, int LX, int LY>
struct LdsFetch {
  const R* s;   // [6][LZ*LX*LY]
  int lv;
  __device__ __forceinline__ R operator()(int comp, int i, int j, int k) const {
    return s[comp * lv + lds_index<LX, LY>(i, j, k)];
  }
};

// Global fetch addressed in a tile's region coordinates.  The origin
// (gz0, gx0, gy0) lies within one period below the grid (periodic z: the
// caller wraps it into [0, nz)), and a region spans at most one period, so a
// single branchless wrap per axis suffices.  Besides the node-wise call, the
// fetch exposes its axes (row offset, column offset, y offset) so that
// gather_axes forms each once per particle; a row outside storage (open z)
// maps to offset 0 and reports !ok, and its weight is then zeroed.
// YC: the tile's region lies inside [0, ny) along y (no wrap), so that a
// stencil's y nodes are consecutive in memory and load as one vector.
template <typename R, bool YC = false>
struct RegionFetch {
  static constexpr bool kYContig = YC;
  const R* const* F;
  Geo g;
  int gz0, gx0, gy0;
  __device__ __forceinline__ int64_t row(int i, bool& ok) const {
    int z = i + gz0;
    if (g.periodic_z) {
      z = wrap_once(z, g.nz);
      ok = true;
    } else {
      ok = z >= -kGuard && z <= g.nz + kGuard;
    }
    return ok ? (int64_t)(z + kGuard) * g.plane : (int64_t)0;
  }
  __device__ __forceinline__ int col(int j) const { return wrap_once(j + gx0, g.nx) * g.ny; }
  __device__ __forceinline__ int dep(int k) const {
    if constexpr (YC) return k + gy0;
    return g.ny > 1 ? wrap_once(k + gy0, g.ny) : 0;
  }
  __device__ __forceinline__ const R* base(int comp, int64_t r) const { return F[comp] + r; }
  __device__ __forceinline__ R operator()(int comp, int i, int j, int k) const {
    bool ok;
    const int64_t r = row(i, ok);
    const R v = base(comp, r)[ok ? col(j) + dep(k) : 0];
    return ok ? v : (R)0;
  }
};

template <class F>
struct HasAxes : std::false_type {};
template <typename R, bool YC>
struct HasAxes<RegionFetch<R, YC>> : std::true_type {};

template <class F>
struct YContig : std::false_type {};
template <typename R>
struct YContig<RegionFetch<R, true>> : std::true_type {};

template <typename R>
struct GlobalFetch {
  const R* const* F;
  Geo g;
  __device__ __forceinline__ R operator()(int comp, int i, int j, int k) const {
    int64_t n = gidx(g, i, j, k);
    return n < 0 ? (R)0 : F[comp][n];
  }
};


// LDS current accumulator of element type A.  FP32 atomic adds on LDS are
// serialised lane by lane on this hardware, FP64 ones are not, so where the
// LDS budget allows the currents accumulate in FP64 (one rounding to the
// working precision at the flush) and every lane adds unconditionally; FP32
// accumulation skips zero addends to keep the serialised lanes few.
template <typename A, int LX, int LY>
struct LdsSink {
  A* s;  // [3][LZ*LX*LY]: Jx Jy Jz
  int lv;
  template <typename R>
  __device__ __forceinline__ void add(int comp, int i, int j, int k, R v) const {
    if constexpr (sizeof(A) == 4) {
      if (v == (R)0) return;
    }
    atomicAdd(&s[comp * lv + lds_index<LX, LY>(i, j, k)], (A)v);
  }
};

// Deterministic mode: currents arrive pre-scaled to fixed-point units (the
// scale is folded into the deposit constants) and are summed as int64, so
// the result does not depend on the order of the atomic adds.
template <int LX, int LY>
struct LdsSinkFx {
  long long* s;  // [3][LZ*LX*LY]
  int lv;
  template <typename R>
  __device__ __forceinline__ void add(int comp, int i, int j, int k, R v) const {
    atomicAdd(reinterpret_cast<unsigned long long*>(&s[comp * lv + lds_index<LX, LY>(i, j, k)]),
              (unsigned long long)to_fixed((double)v));
  }
};

// Accumulator type of the tiled kernel's LDS currents: FP64, except 3D with
// staged fields, which keeps the working precision so that fields and
// currents fit in LDS; deterministic mode: int64 fixed point.
template <typename R, int DIM, bool DET, bool STAGE = true>
using LdsAcc = typename std::conditional<
    DET, long long,
    typename std::conditional<DIM == 2 || !STAGE, double, R>::type>::type;

template <typename A, int LX, int LY, bool DET>
using LdsSinkT = typename std::conditional<DET, LdsSinkFx<LX, LY>, LdsSink<A, LX, LY>>::type;

template <typename R>
struct GlobalSink {
  Ovf<R> o;
  Geo g;
  __device__ __forceinline__ void add(int comp, int i, int j, int k, R v) const {
    if (v == (R)0) return;
    int64_t n = gidx(g, i, j, k);
    if (n >= 0) atomicAdd(&o.J[comp][n], v);
  }
};

template <typename R>
struct GlobalSinkFx {
  Ovf<R> o;
  Geo g;
  __device__ __forceinline__ void add(int comp, int i, int j, int k, R v) const {
    if (v == (R)0) return;
    int64_t n = gidx(g, i, j, k);
    if (n >= 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(&o.Jq[comp][n]),
                (unsigned long long)to_fixed((double)v));
  }
};

// --------------------------------------------------------------------------
// Gather: each component interpolated from its own staggered lattice with the
// deposit's shape (momentum-conserving gather).  bc = the particle's cell in
// the fetcher's frame, p its absolute position.
// --------------------------------------------------------------------------
// Fetches that read global memory: their stencil values are all loaded
// before any is used (LDS fetches keep the interleaved form).
template <class F>
struct LoadsFirst : std::false_type {};
template <typename R>
struct LoadsFirst<GlobalFetch<R>> : std::true_type {};

template <typename R, int DIM, int ORDER, class F>
__device__ __forceinline__ R interp(const F& f, int comp, int bz, const R* wz, int bx, const R* wx,
                                    int by, const R* wy) {
  if constexpr (LoadsFirst<F>::value) {
    constexpr int N = ORDER + 1, NY = DIM == 3 ? N : 1;
    R v[N][N][NY];
#pragma unroll
    for (int a = 0; a < N; a++)
#pragma unroll
      for (int b = 0; b < N; b++)
#pragma unroll
        for (int c = 0; c < NY; c++) v[a][b][c] = f(comp, bz + a, bx + b, DIM == 3 ? by + c : 0);
    R acc = (R)0;
#pragma unroll
    for (int a = 0; a < N; a++) {
      R rowz = (R)0;
#pragma unroll
      for (int b = 0; b < N; b++) {
        if (DIM == 3) {
          R cy = (R)0;
#pragma unroll
          for (int c = 0; c < N; c++) cy += v[a][b][c] * wy[c];
          rowz += cy * wx[b];
        } else {
          rowz += v[a][b][0] * wx[b];
        }
      }
      acc += rowz * wz[a];
    }
    return acc;
  }
  R acc = (R)0;
#pragma unroll
  for (int a = 0; a <= ORDER; a++) {
    R rowz = (R)0;
#pragma unroll
    for (int b = 0; b <= ORDER; b++) {
      if (DIM == 3) {
        R cy = (R)0;
#pragma unroll
        for (int c = 0; c <= ORDER; c++) cy += f(comp, bz + a, bx + b, by + c) * wy[c];
        rowz += cy * wx[b];
      } else {
        rowz += f(comp, bz + a, bx + b, 0) * wx[b];
      }
    }
    acc += rowz * wz[a];
  }
  return acc;
}

// Gather through a fetch that exposes its axes: per staggering set (integer,
// half) and axis, the node offsets are formed once, then each component's
// stencil reads base(comp, row)[col + dep].
// All the stencil's node values are loaded before any is used, so that the
// loads of one component are in flight together (from L2 or HBM, each takes
// hundreds of cycles).
template <typename R, int DIM, int ORDER, class F>
__device__ __forceinline__ R interp_axes(const F& f, int comp, const int64_t* zr, const R* wz,
                                         const int* xc, const R* wx, const int* yc,
                                         const R* wy) {
  constexpr int N = ORDER + 1, NY = DIM == 3 ? N : 1;
  R v[N][N][NY];
#pragma unroll
  for (int a = 0; a < N; a++) {
    const R* rp = f.base(comp, zr[a]);
#pragma unroll
    for (int b = 0; b < N; b++) {
      if constexpr (DIM == 3 && YContig<F>::value) {
        // consecutive y nodes: one multi-dword load (element alignment only)
        __builtin_memcpy(&v[a][b][0], rp + xc[b] + yc[0], sizeof(R) * NY);
      } else {
#pragma unroll
        for (int c = 0; c < NY; c++) v[a][b][c] = rp[xc[b] + (DIM == 3 ? yc[c] : 0)];
      }
    }
  }
  R acc = (R)0;
#pragma unroll
  for (int a = 0; a < N; a++) {
    R rowz = (R)0;
#pragma unroll
    for (int b = 0; b < N; b++) {
      if (DIM == 3) {
        R cy = (R)0;
#pragma unroll
        for (int c = 0; c < N; c++) cy += v[a][b][c] * wy[c];
        rowz += cy * wx[b];
      } else {
        rowz += v[a][b][0] * wx[b];
      }
    }
    acc += rowz * wz[a];
  }
  return acc;
}

// Galerkin (energy-conserving) form: every half-lattice weight set replaced
// by the shape of one order lower on the same nodes (a component staggered
// along an axis takes the reduced shape along that axis).
template <typename R, int ORDER>
__device__ __forceinline__ void galerkin_half(bool gk, R o, R w[ORDER + 1]) {
  if (gk) shape_half_reduced<R, ORDER>(o, w);
}

template <typename R, int DIM, int ORDER, class F>
__device__ __forceinline__ void gather_axes(const F& f, const int bc[3], const Pos<R>& p, R E[3],
                                            R B[3], bool gk) {
  R wz[2][ORDER + 1], wx[2][ORDER + 1], wy[2][ORDER + 1];
  int64_t zr[2][ORDER + 1];
  int xc[2][ORDER + 1], yc[2][ORDER + 1];
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int bz = shape<R, ORDER>(p.c[0], p.o[0], h, wz[h]) - p.c[0] + bc[0];
    const int bx = shape<R, ORDER>(p.c[1], p.o[1], h, wx[h]) - p.c[1] + bc[1];
    if (h == 1) {
      galerkin_half<R, ORDER>(gk, p.o[0], wz[h]);
      galerkin_half<R, ORDER>(gk, p.o[1], wx[h]);
    }
#pragma unroll
    for (int a = 0; a <= ORDER; a++) {
      bool ok;
      zr[h][a] = f.row(bz + a, ok);
      wz[h][a] = ok ? wz[h][a] : (R)0;
      xc[h][a] = f.col(bx + a);
    }
    if (DIM == 3) {
      const int by = shape<R, ORDER>(p.c[2], p.o[2], h, wy[h]) - p.c[2] + bc[2];
      if (h == 1) galerkin_half<R, ORDER>(gk, p.o[2], wy[h]);
#pragma unroll
      for (int c = 0; c <= ORDER; c++) yc[h][c] = f.dep(by + c);
    } else {
#pragma unroll
      for (int c = 0; c <= ORDER; c++) {
        wy[h][c] = (R)0;
        yc[h][c] = 0;
      }
    }
  }
  // staggering (z, x, y): Ex (0,h,0) Ey (0,0,h) Ez (h,0,0) Bx (h,0,h) By (h,h,0) Bz (0,h,h)
  E[0] = interp_axes<R, DIM, ORDER>(f, 0, zr[0], wz[0], xc[1], wx[1], yc[0], wy[0]);
  E[1] = interp_axes<R, DIM, ORDER>(f, 1, zr[0], wz[0], xc[0], wx[0], yc[1], wy[1]);
  E[2] = interp_axes<R, DIM, ORDER>(f, 2, zr[1], wz[1], xc[0], wx[0], yc[0], wy[0]);
  B[0] = interp_axes<R, DIM, ORDER>(f, 3, zr[1], wz[1], xc[0], wx[0], yc[1], wy[1]);
  B[1] = interp_axes<R, DIM, ORDER>(f, 4, zr[1], wz[1], xc[1], wx[1], yc[0], wy[0]);
  B[2] = interp_axes<R, DIM, ORDER>(f, 5, zr[0], wz[0], xc[1], wx[1], yc[1], wy[1]);
}

template <typename R, int DIM, int ORDER, class F>
__device__ __forceinline__ void gather_nodes(const F& f, const int bc[3], const Pos<R>& p,
                                             R E[3], R B[3], bool gk) {
  R wz0[ORDER + 1], wz1[ORDER + 1], wx0[ORDER + 1], wx1[ORDER + 1];
  R wy0[ORDER + 1], wy1[ORDER + 1];
  int z0 = shape<R, ORDER>(p.c[0], p.o[0], 0, wz0) - p.c[0] + bc[0];
  int z1 = shape<R, ORDER>(p.c[0], p.o[0], 1, wz1) - p.c[0] + bc[0];
  int x0 = shape<R, ORDER>(p.c[1], p.o[1], 0, wx0) - p.c[1] + bc[1];
  int x1 = shape<R, ORDER>(p.c[1], p.o[1], 1, wx1) - p.c[1] + bc[1];
  galerkin_half<R, ORDER>(gk, p.o[0], wz1);
  galerkin_half<R, ORDER>(gk, p.o[1], wx1);
  int y0 = 0, y1 = 0;
  if (DIM == 3) {
    y0 = shape<R, ORDER>(p.c[2], p.o[2], 0, wy0) - p.c[2] + bc[2];
    y1 = shape<R, ORDER>(p.c[2], p.o[2], 1, wy1) - p.c[2] + bc[2];
    galerkin_half<R, ORDER>(gk, p.o[2], wy1);
  }
  // staggering (z, x, y): Ex (0,h,0) Ey (0,0,h) Ez (h,0,0) Bx (h,0,h) By (h,h,0) Bz (0,h,h)
  E[0] = interp<R, DIM, ORDER>(f, 0, z0, wz0, x1, wx1, y0, wy0);
  E[1] = interp<R, DIM, ORDER>(f, 1, z0, wz0, x0, wx0, y1, wy1);
  E[2] = interp<R, DIM, ORDER>(f, 2, z1, wz1, x0, wx0, y0, wy0);
  B[0] = interp<R, DIM, ORDER>(f, 3, z1, wz1, x0, wx0, y1, wy1);
  B[1] = interp<R, DIM, ORDER>(f, 4, z1, wz1, x1, wx1, y0, wy0);
  B[2] = interp<R, DIM, ORDER>(f, 5, z0, wz0, x1, wx1, y1, wy1);
}

template <typename R, int DIM, int ORDER, class F>
__device__ __forceinline__ void gather(const F& f, const int bc[3], const Pos<R>& p, R E[3],
                                       R B[3], bool gk) {
  if constexpr (HasAxes<F>::value) gather_axes<R, DIM, ORDER>(f, bc, p, E, B, gk);
  else gather_nodes<R, DIM, ORDER>(f, bc, p, E, B, gk);
}

// --------------------------------------------------------------------------
// Esirkepov stencil along one axis: old and new shape factors of the charge
// lattice placed on NS = ORDER + 2 nodes starting at bs.
// --------------------------------------------------------------------------
template <typename R, int ORDER>
__device__ __forceinline__ void place(bool shifted, const R* w, R* S) {
  constexpr int NS = ORDER + 2;
#pragma unroll
  for (int m = 0; m < NS; m++) {
    R lo = m <= ORDER ? w[m < ORDER + 1 ? m : 0] : (R)0;
    R hi = m >= 1 ? w[m >= 1 ? m - 1 : 0] : (R)0;
    S[m] = shifted ? hi : lo;
  }
}

template <typename R, int ORDER>
__device__ __forceinline__ int esk_axis(int c0, R o0, int c1, R o1, R* S0, R* dS) {
  constexpr int NS = ORDER + 2;
  R w0[ORDER + 1], w1[ORDER + 1], S1[NS];
  int b0 = shape<R, ORDER>(c0, o0, 0, w0);
  int b1 = shape<R, ORDER>(c1, o1, 0, w1);
  int bs = b0 < b1 ? b0 : b1;
  place<R, ORDER>(b0 != bs, w0, S0);
  place<R, ORDER>(b1 != bs, w1, S1);
#pragma unroll
  for (int m = 0; m < NS; m++) dS[m] = S1[m] - S0[m];
  return bs;
}

// --------------------------------------------------------------------------
// Deposit of one electron (charge -w) moving e0 -> e1 and of its partner
// (charge +w) moving i0 -> i1 along z.  When the partner's stencil lies
// inside the electron's, both W patterns are combined before the prefix sums,
// so an unperturbed pair deposits exactly zero.
// --------------------------------------------------------------------------
template <typename R, int ORDER, class Snk>
__device__ __forceinline__ void deposit2d(const StepK<R>& P, const Snk& snk, const int bc[3],
                                          const Pos<R>& e0, const Pos<R>& e1, const Pos<R>& i0,
                                          const Pos<R>& i1, R w, R vy, bool with_ion = true) {
  constexpr int NS = ORDER + 2;
  R S0z[NS], dSz[NS], S0x[NS], dSx[NS];
  int bz = esk_axis<R, ORDER>(e0.c[0], e0.o[0], e1.c[0], e1.o[0], S0z, dSz);
  int bx = esk_axis<R, ORDER>(e0.c[1], e0.o[1], e1.c[1], e1.o[1], S0x, dSx);
  const int rz = bc[0] + (bz - e0.c[0]), rx = bc[1] + (bx - e0.c[1]);
  // partner: moves along z only (with_ion = false: the caller deposits it)
  R I0z[NS], dIz[NS], Ix[NS];
  bool ion = P.ion_moves && with_ion;
  bool comb = false;
  int ibz = 0, ibx = 0;
  if (ion) {
    ibz = esk_axis<R, ORDER>(i0.c[0], i0.o[0], i1.c[0], i1.o[0], I0z, dIz);
    R wx[ORDER + 1];
    ibx = shape<R, ORDER>(i0.c[1], i0.o[1], 0, wx);
    int ox = ibx - bx;
    comb = (ibz == bz) && (ox == 0 || ox == 1);
    place<R, ORDER>(ox == 1, wx, Ix);
  }
  // Jz: prefix along z of kz w (We - Wi), We = dSz (S0x + dSx/2), Wi = dIz Ix
  const R kz = P.kj[0] * w;
#pragma unroll
  for (int b = 0; b < NS; b++) {
    R fx = S0x[b] + (R)0.5 * dSx[b];
    R acc = (R)0;
#pragma unroll
    for (int a = 0; a < NS - 1; a++) {
      R We = dSz[a] * fx;
      R Wi = comb ? dIz[a] * Ix[b] : (R)0;
      acc += kz * (We - Wi);
      snk.add(2, rz + a, rx + b, 0, acc);
    }
  }
  if (ion && !comb) {
    const int irz = bc[0] + (ibz - e0.c[0]), irx = bc[1] + (ibx - e0.c[1]);
    R wx[ORDER + 1];
    shape<R, ORDER>(i0.c[1], i0.o[1], 0, wx);
#pragma unroll
    for (int b = 0; b <= ORDER; b++) {
      R acc = (R)0;
#pragma unroll
      for (int a = 0; a < NS - 1; a++) {
        acc -= kz * dIz[a] * wx[b];
        snk.add(2, irz + a, irx + b, 0, acc);
      }
    }
  }
  // Jx: prefix along x of kx w We, We = dSx (S0z + dSz/2)
  const R kx = P.kj[1] * w;
#pragma unroll
  for (int a = 0; a < NS; a++) {
    R fz = S0z[a] + (R)0.5 * dSz[a];
    R acc = (R)0;
#pragma unroll
    for (int b = 0; b < NS - 1; b++) {
      acc += kx * dSx[b] * fz;
      snk.add(0, rz + a, rx + b, 0, acc);
    }
  }
  // Jy (out of plane): q w vy Wy / (dz dx), Wy the time-averaged shape product
  if (vy != (R)0) {
    const R ky = -P.ky2d * w * vy;
#pragma unroll
    for (int a = 0; a < NS; a++)
#pragma unroll
      for (int b = 0; b < NS; b++) {
        R wy = S0z[a] * S0x[b] + (R)0.5 * (dSz[a] * S0x[b] + S0z[a] * dSx[b]) +
               dSz[a] * dSx[b] * (R)(1.0 / 3.0);
        snk.add(1, rz + a, rx + b, 0, ky * wy);
      }
  }
}

// --------------------------------------------------------------------------
// Pair deposit, linear shape, 2D.  The electron sits at its partner's position
// plus xi; with u = o + xi (o the partner's offset in its cell) the linear
// shape factors of nodes k = -1..2 of the partner's cell differ from the
// partner's by
//   u < 0:      dS = (-u, 2 o + xi, -o, 0)
//   0 <= u < 1: dS = (0, -xi, xi, 0)
//   1 <= u < 2: dS = (0, o - 1, 2 (1 - o) - xi, (o - 1) + xi)
// (partner weights (0, 1 - o, o, 0)), so electron minus partner is formed
// from xi and exact offset distances only, never from two nearly equal
// positions.  Only Jz carries the pair difference (the partner moves along z
// only); Jx and Jy are the electron's own and use its plain stencil.
// --------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ bool lin_pair(R o, R xi, R Si[4], R dS[4]) {
  R u = o + xi;
  bool lo = u < (R)0, hi = u >= (R)1;
  R om1 = o - (R)1;
  Si[0] = (R)0;
  Si[1] = (R)1 - o;
  Si[2] = o;
  Si[3] = (R)0;
  dS[0] = lo ? -u : (R)0;
  dS[1] = lo ? (o + o) + xi : (hi ? om1 : -xi);
  dS[2] = lo ? -o : (hi ? (R)-2 * om1 - xi : xi);
  dS[3] = hi ? om1 + xi : (R)0;
  return u >= (R)-1 && u < (R)2;
}

// shift a 4-node array by s in {0, 1} into a 4-node window (entry 3 drops)
template <typename R>
__device__ __forceinline__ R at4(const R a[4], int s, int m) {
  R v0 = m < 4 ? a[m < 4 ? m : 0] : (R)0;
  R v1 = m >= 1 ? a[m >= 1 ? m - 1 : 0] : (R)0;
  return s ? v1 : v0;
}

template <typename R, class Snk>
__device__ __forceinline__ bool deposit2d_pair(const StepK<R>& P, const Snk& snk, const int bc[3],
                                               const Pos<R>& e0, const Pos<R>& e1,
                                               const Pos<R>& i0, const Pos<R>& i1,
                                               const R xi0[3], const R xi1[3], R w, R vy) {
  // z: partner old / new, electron = partner + xi
  R Sa[4], da[4], Sb[4], db[4], Sx[4], dx0[4], dx1[4];
  bool ok = lin_pair(i0.o[0], xi0[0], Sa, da);
  ok &= lin_pair(i1.o[0], xi1[0], Sb, db);
  ok &= lin_pair(i0.o[1], xi0[1], Sx, dx0);
  R unused[4];
  ok &= lin_pair(i0.o[1], xi1[1], unused, dx1);
  const int W = min(i0.c[0], i1.c[0]) - 1;
  const int s0 = i0.c[0] - 1 - W, s1 = i1.c[0] - 1 - W;  // each 0 or 1
  // a shifted array loses its top node, which must then be empty
  ok &= !(s0 && da[3] != (R)0) && !(s1 && db[3] != (R)0);
  ok &= (unsigned)s0 <= 1u && (unsigned)s1 <= 1u;
  if (!ok) return false;
  R dSi[4], eps[4];
#pragma unroll
  for (int m = 0; m < 4; m++) {
    dSi[m] = P.ion_moves ? at4(Sb, s1, m) - at4(Sa, s0, m) : (R)0;
    eps[m] = at4(db, s1, m) - at4(da, s0, m);
  }
  const int rz = bc[0] + (W - e0.c[0]), rx = bc[1] + (i0.c[1] - 1 - e0.c[1]);
  const R kz = P.kj[0] * w;
  // Jz(a + 1/2, b) = kz sum_{a' <= a} (dSi eta + eps fx_e) = kz (CSi[a] eta[b] + Ceps[a] fxe[b])
  R CSi[3], Ce[3];
  CSi[0] = kz * dSi[0];
  Ce[0] = kz * eps[0];
#pragma unroll
  for (int a2 = 1; a2 < 3; a2++) {
    CSi[a2] = CSi[a2 - 1] + kz * dSi[a2];
    Ce[a2] = Ce[a2 - 1] + kz * eps[a2];
  }
  // A column is all zeros when eta = 0 and Ce (or fxe) = 0: a pair whose
  // electron keeps its offset from the partner deposits nothing at all.  The
  // tests are per lane, so a wave whose lanes all have zeros skips the column.
  const bool ce_any = Ce[0] != (R)0 || Ce[1] != (R)0 || Ce[2] != (R)0;
#pragma unroll
  for (int b = 0; b < 4; b++) {
    const R eta = (R)0.5 * (dx0[b] + dx1[b]);
    const R fxe = Sx[b] + eta;
    if (eta != (R)0 || (ce_any && fxe != (R)0)) {
#pragma unroll
      for (int a2 = 0; a2 < 3; a2++)
        snk.add(2, rz + a2, rx + b, 0, CSi[a2] * eta + Ce[a2] * fxe);
    }
  }
  // Jx, Jy: the electron alone, on its own 3-node stencil.
  //   Jx(a, b + 1/2) = fz[a] * kx sum_{b' <= b} dSx[b'],  fz = S0z + dSz / 2
  //   Wy = S0z S0x + (dSz S0x + S0z dSx) / 2 + dSz dSx / 3 = fz fx + dSz dSx / 12
  constexpr int NS = 3;
  R S0z[NS], dSz[NS], S0x[NS], dSx[NS];
  int bz = esk_axis<R, 1>(e0.c[0], e0.o[0], e1.c[0], e1.o[0], S0z, dSz);
  int bx = esk_axis<R, 1>(e0.c[1], e0.o[1], e1.c[1], e1.o[1], S0x, dSx);
  const int ez = bc[0] + (bz - e0.c[0]), ex = bc[1] + (bx - e0.c[1]);
  const R kx = P.kj[1] * w;
  R fz[NS], fx[NS];
#pragma unroll
  for (int m = 0; m < NS; m++) {
    fz[m] = S0z[m] + (R)0.5 * dSz[m];
    fx[m] = S0x[m] + (R)0.5 * dSx[m];
  }
  const R cx0 = kx * dSx[0], cx1 = cx0 + kx * dSx[1];
  if (cx0 != (R)0) {  // zero without motion along x (as cx1)
#pragma unroll
    for (int a2 = 0; a2 < NS; a2++) snk.add(0, ez + a2, ex + 0, 0, fz[a2] * cx0);
  }
  if (cx1 != (R)0) {
#pragma unroll
    for (int a2 = 0; a2 < NS; a2++) snk.add(0, ez + a2, ex + 1, 0, fz[a2] * cx1);
  }
  if (vy != (R)0) {
    const R ky = -P.ky2d * w * vy;
    const R ky12 = ky * (R)(1.0 / 12.0);
#pragma unroll
    for (int a2 = 0; a2 < NS; a2++) {
      const R za = ky * fz[a2], zb = ky12 * dSz[a2];
#pragma unroll
      for (int b = 0; b < NS; b++) snk.add(1, ez + a2, ex + b, 0, za * fx[b] + zb * dSx[b]);
    }
  }
  return true;
}

template <typename R>
__device__ __forceinline__ R wmix(R s0a, R dsa, R s0b, R dsb) {
  return s0a * s0b + (R)0.5 * (dsa * s0b + s0a * dsb) + dsa * dsb * (R)(1.0 / 3.0);
}

template <typename R, int ORDER, class Snk>
__device__ __forceinline__ void deposit3d(const StepK<R>& P, const Snk& snk, const int bc[3],
                                          const Pos<R>& e0, const Pos<R>& e1, const Pos<R>& i0,
                                          const Pos<R>& i1, R w, bool with_ion = true) {
  constexpr int NS = ORDER + 2;
  R S0z[NS], dSz[NS], S0x[NS], dSx[NS], S0y[NS], dSy[NS];
  int bz = esk_axis<R, ORDER>(e0.c[0], e0.o[0], e1.c[0], e1.o[0], S0z, dSz);
  int bx = esk_axis<R, ORDER>(e0.c[1], e0.o[1], e1.c[1], e1.o[1], S0x, dSx);
  int by = esk_axis<R, ORDER>(e0.c[2], e0.o[2], e1.c[2], e1.o[2], S0y, dSy);
  const int rz = bc[0] + (bz - e0.c[0]), rx = bc[1] + (bx - e0.c[1]),
            ry = bc[2] + (by - e0.c[2]);
  R I0z[NS], dIz[NS], Ix[NS], Iy[NS];
  bool ion = P.ion_moves && with_ion, comb = false;
  int ibz = 0, ibx = 0, iby = 0;
  R wxi[ORDER + 1], wyi[ORDER + 1];
  if (ion) {
    ibz = esk_axis<R, ORDER>(i0.c[0], i0.o[0], i1.c[0], i1.o[0], I0z, dIz);
    ibx = shape<R, ORDER>(i0.c[1], i0.o[1], 0, wxi);
    iby = shape<R, ORDER>(i0.c[2], i0.o[2], 0, wyi);
    int ox = ibx - bx, oy = iby - by;
    comb = (ibz == bz) && (ox == 0 || ox == 1) && (oy == 0 || oy == 1);
    place<R, ORDER>(ox == 1, wxi, Ix);
    place<R, ORDER>(oy == 1, wyi, Iy);
  }
  const R kz = P.kj[0] * w, kx = P.kj[1] * w, ky = P.kj[2] * w;
  // Columns of the stencil whose values are all zero are skipped: a wave
  // whose lanes all hold zeros for a column issues none of its LDS adds.  A
  // pair whose electron keeps its offset from the partner (co-located, moving
  // with it) gives exact zeros: the partner's term uses the same products as
  // the electron's (dIz (Ix Iy) against dSz f with f = S0x S0y), and J_x, J_y
  // vanish without x, y motion.
#pragma unroll
  for (int b = 0; b < NS; b++)
#pragma unroll
    for (int c = 0; c < NS; c++) {
      const R f = wmix(S0x[b], dSx[b], S0y[c], dSy[c]);
      const R fi = comb ? Ix[b] * Iy[c] : (R)0;
      R v[NS - 1];
      R acc = (R)0;
      bool any = false;
#pragma unroll
      for (int a = 0; a < NS - 1; a++) {
        const R Wi = comb ? dIz[a] * fi : (R)0;
        acc += kz * (dSz[a] * f - Wi);
        v[a] = acc;
        any = any || acc != (R)0;
      }
      if (any) {
#pragma unroll
        for (int a = 0; a < NS - 1; a++) snk.add(2, rz + a, rx + b, ry + c, v[a]);
      }
    }
  if (ion && !comb) {
    const int irz = bc[0] + (ibz - e0.c[0]), irx = bc[1] + (ibx - e0.c[1]),
              iry = bc[2] + (iby - e0.c[2]);
#pragma unroll
    for (int b = 0; b <= ORDER; b++)
#pragma unroll
      for (int c = 0; c <= ORDER; c++) {
        R acc = (R)0;
#pragma unroll
        for (int a = 0; a < NS - 1; a++) {
          acc -= kz * dIz[a] * wxi[b] * wyi[c];
          snk.add(2, irz + a, irx + b, iry + c, acc);
        }
      }
  }
  bool mx = false, my = false;  // any motion along x, y
#pragma unroll
  for (int m = 0; m < NS; m++) {
    mx = mx || dSx[m] != (R)0;
    my = my || dSy[m] != (R)0;
  }
  if (mx) {
#pragma unroll
    for (int a = 0; a < NS; a++)
#pragma unroll
      for (int c = 0; c < NS; c++) {
        R f = wmix(S0z[a], dSz[a], S0y[c], dSy[c]);
        R acc = (R)0;
#pragma unroll
        for (int b = 0; b < NS - 1; b++) {
          acc += kx * dSx[b] * f;
          snk.add(0, rz + a, rx + b, ry + c, acc);
        }
      }
  }
  if (my) {
#pragma unroll
    for (int a = 0; a < NS; a++)
#pragma unroll
      for (int b = 0; b < NS; b++) {
        R f = wmix(S0z[a], dSz[a], S0x[b], dSx[b]);
        R acc = (R)0;
#pragma unroll
        for (int c = 0; c < NS - 1; c++) {
          acc += ky * dSy[c] * f;
          snk.add(1, rz + a, rx + b, ry + c, acc);
        }
      }
  }
}

// --------------------------------------------------------------------------
// One particle step after its positions are known: gather at e0, push, move,
// deposit, decide removal.  Returns the new displacement through xi.
// --------------------------------------------------------------------------
// Called with the gathered fields before the push (the adjoint seeds them).
struct NoHook {
  template <typename R>
  __device__ __forceinline__ void operator()(R*, R*) const {}
};

template <typename R, int DIM, int ORDER, class F, class Snk, class Hook = NoHook>
__device__ __forceinline__ bool particle_step(const StepK<R>& P, const F& fetch, const Snk& snk,
                                              const int bc[3], const Pos<R>& e0,
                                              const Pos<R>& i0, const Pos<R>& i1, R xi[3],
                                              R du[3], R w, const Hook& hook = Hook(),
                                              bool near = true) {
  R E[3], B[3], dv[3], gam;
  gather<R, DIM, ORDER>(fetch, bc, e0, E, B, P.galerkin != 0);
  hook(E, B);
  boris_split(P.push, E, B, du, dv, gam);
  const R xi_old[3] = {xi[0], xi[1], xi[2]};
  // position axes (z, x, y) <- velocity components (z, x, y) = dv[2], dv[0], dv[1]
  xi[0] += dv[2] * P.dtd[0];
  xi[1] += dv[0] * P.dtd[1];
  if (DIM == 3) xi[2] += dv[1] * P.dtd[2];
  Pos<R> e1 = add_xi<R, DIM>(i1, xi);
  if (DIM == 2) {
    bool done = false;
    // near = false: the partner is out of the sink's reach and the caller
    // deposits it (partner_far); the electron deposits alone
    if constexpr (ORDER == 1)
      if (near) done = deposit2d_pair<R>(P, snk, bc, e0, e1, i0, i1, xi_old, xi, w, dv[1]);
    if (!done) deposit2d<R, ORDER>(P, snk, bc, e0, e1, i0, i1, w, dv[1], near);
  } else {
    deposit3d<R, ORDER>(P, snk, bc, e0, e1, i0, i1, w, near);
  }
  if (!P.remove) return false;
  // outside [-lim, nz + lim] along z, for both members of the pair
  const int lo = -P.lim - 1, hi = P.g.nz + P.lim;
  bool eo = e1.c[0] <= lo || e1.c[0] > hi || (e1.c[0] == hi && e1.o[0] > (R)0);
  bool io = i1.c[0] <= lo || i1.c[0] > hi || (i1.c[0] == hi && i1.o[0] > (R)0);
  return eo && io;
}

// Current of a partner deposited on its own, at absolute nodes of the
// overflow grid: it moves along z only, so its Esirkepov current is Jz alone
// (the separate-stencil terms of deposit2d / deposit3d, in the same order).
// Its nodes lie within a node of its birth column (and row of y), so one
// branchless wrap places them; rows outside storage (open z) are dropped.
template <typename R, int DIM, int ORDER, bool DET>
__device__ __forceinline__ void partner_far(const StepK<R>& P, const Ovf<R>& O, const Pos<R>& i0,
                                            const Pos<R>& i1, R w) {
  if (!P.ion_moves) return;
  const Geo& g = P.g;
  constexpr int NS = ORDER + 2;
  constexpr int NY = DIM == 3 ? ORDER + 1 : 1;
  R I0z[NS], dIz[NS], wx[ORDER + 1], wy[ORDER + 1];
  const int ibz = esk_axis<R, ORDER>(i0.c[0], i0.o[0], i1.c[0], i1.o[0], I0z, dIz);
  const int ibx = shape<R, ORDER>(i0.c[1], i0.o[1], 0, wx);
  const int iby = DIM == 3 ? shape<R, ORDER>(i0.c[2], i0.o[2], 0, wy) : 0;
  const R kz = P.kj[0] * w;
#pragma unroll
  for (int b = 0; b <= ORDER; b++)
#pragma unroll
    for (int c = 0; c < NY; c++) {
      const int j = wrap_once(ibx + b, g.nx);
      const int k = DIM == 3 ? wrap_once(iby + c, g.ny) : 0;
      R acc = (R)0;
#pragma unroll
      for (int a = 0; a < NS - 1; a++) {
        if (DIM == 3) acc -= kz * dIz[a] * wx[b] * wy[c];
        else acc -= kz * dIz[a] * wx[b];
        int i = ibz + a;
        if (g.periodic_z) i = wrapi(i, g.nz);  // absolute rows carry the whole drift
        else if (i < -kGuard || i > g.nz + kGuard) continue;
        if (acc == (R)0) continue;
        const int64_t n = ((int64_t)(i + kGuard) * g.nx + j) * g.ny + k;
        if constexpr (DET)
          atomicAdd(reinterpret_cast<unsigned long long*>(&O.Jq[2][n]),
                    (unsigned long long)to_fixed((double)acc));
        else
          atomicAdd(&O.J[2][n], acc);
      }
    }
}

template <typename R>
__device__ __forceinline__ void load_state(const PSoA<R>& S, int p, R xi[3], R du[3], R& w) {
  xi[0] = S.xi[0][p];
  xi[1] = S.xi[1][p];
  xi[2] = S.xi[2] ? S.xi[2][p] : (R)0;
  du[0] = S.du[0][p];
  du[1] = S.du[1][p];
  du[2] = S.du[2][p];
  w = S.w[p];
}

template <typename R, int DIM>
__device__ __forceinline__ void store_state(const PSoA<R>& S, int p, const R xi[3], const R du[3],
                                            bool dead) {
  S.xi[0][p] = xi[0];
  S.xi[1][p] = xi[1];
  if (DIM == 3) S.xi[2][p] = xi[2];
  S.du[0][p] = du[0];
  S.du[1][p] = du[1];
  S.du[2][p] = du[2];
  if (dead) S.id[p] = -1;
}

// Row range of a particle's stencils (for the overflow fold).
template <typename R, int ORDER>
__device__ __forceinline__ void note_rows(const Ovf<R>& o, const Geo& g, int ce, int ci) {
  if (g.periodic_z) {
    atomicMin(&o.rows[0], 0);
    atomicMax(&o.rows[1], g.nz);
    return;
  }
  int lo = (ce < ci ? ce : ci) - ORDER - 1;
  int hi = (ce > ci ? ce : ci) + ORDER + 2;
  atomicMin(&o.rows[0], lo);
  atomicMax(&o.rows[1], hi);
}

// --------------------------------------------------------------------------
// Global path: the unsorted tail [first, counts[0]) plus the stragglers the
// tiled kernel listed (particles whose stencil left their tile's region), or
// every slot when the grid is too small to tile.  Fields are read and the
// current is accumulated in global memory (the overflow sink).
// --------------------------------------------------------------------------
template <typename R, int DIM, int ORDER, bool DET>
__global__ __launch_bounds__(256) void k_gpd_global(StepK<R> P, Fields<R> F, PSoA<R> S, Ovf<R> O,
                                                    const int* counts, int from_sorted,
                                                    const int* strag, const int* nstrag) {
  const int first = from_sorted ? counts[1] : 0;
  const int ntail = counts[0] - first;
  const int total = ntail + (strag ? *nstrag : 0);
  GlobalFetch<R> f{(const R* const*)F.F, P.g};
  typename std::conditional<DET, GlobalSinkFx<R>, GlobalSink<R>>::type sk{O, P.g};
  // An injected tail is whole lattice columns, the ppc slots of a cell in a
  // row: it is taken slot-major (thread q: cell q mod m, slot q / m), so that
  // the lanes of a wave deposit around distinct cells rather than piling
  // their atomics onto the nodes of one cell.
  const int ppc = P.L.ppc;
  const bool il = from_sorted && ppc > 1 && ntail % ppc == 0;
  const int m = il ? ntail / ppc : 1;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
    int p;
    if (q < ntail) {
      const int qs = q / m;
      p = first + (il ? (q - qs * m) * ppc + qs : q);
    } else {
      p = strag[q - ntail];
    }
    const int id = S.id[p];
    if (id < 0) continue;
    R xi[3], du[3], w;
    load_state(S, p, xi, du, w);
    Birth b = decode_id(P.L, id);
    R r[3];
    birth_offsets<R, DIM>(P.L, id, r);
    Pos<R> i0 = ion_at<R, DIM>(b, r, P.D0);
    Pos<R> i1 = ion_at<R, DIM>(b, r, P.D1);
    Pos<R> e0 = add_xi<R, DIM>(i0, xi);
    int bc[3] = {e0.c[0], e0.c[1], e0.c[2]};
    note_rows<R, ORDER>(O, P.g, e0.c[0], i0.c[0]);
    bool dead = particle_step<R, DIM, ORDER>(P, f, sk, bc, e0, i0, i1, xi, du, w);
    store_state<R, DIM>(S, p, xi, du, dead);
  }
}

// --------------------------------------------------------------------------
// Tiled path.  One workgroup per co-moving tile of TZ x TX [x TY] cells.  The
// tile's E, B and a zeroed J accumulator are staged in LDS over the tile plus
// a margin of EXC cells of peculiar excursion, one row of drift and the
// stencil reach; each particle of the tile gathers from LDS and deposits with
// LDS atomics; the J region is then stored whole to the tile's scratch slot,
// to be folded into the grid by the filter kernel.  A particle whose own
// stencil would leave the region is appended to the straggler list instead
// and is advanced by the global path in the same step; one whose partner
// lies out of reach deposits the partner's current to the overflow grid.
// --------------------------------------------------------------------------
struct TileK {
  const int* start;  // particle range of tile t: [start[t], start[t+1])
  const int* order;  // dispatch order (largest first), or null: XCD-aware grid order
  int ntiles, ntx, nty;
  int zc0;           // first co-moving z cell of tile row 0
  int* strag;        // straggler slots
  int* nstrag;       // their count
  unsigned* box;     // 3D: per tile, the box of its region's nonzero nodes
};

// Region of a tile: its cells, the excursion margin EXC on each side, one row
// of plasma drift along z, and the stencil reach HLO below / HHI above a cell
// (the 4-node pair window reaches two nodes below the partner's cell when the
// partner crosses a cell, and one spare node above).
template <int DIM, int ORDER, int TZ, int TX, int TY, int EXC>
struct TileGeom {
  static constexpr int HLO = ORDER + 1;
  static constexpr int HHI = ORDER + 2;
  static constexpr int LZ = TZ + 2 * EXC + 1 + HLO + HHI;
  static constexpr int LX = TX + 2 * EXC + HLO + HHI;
  static constexpr int LY = DIM == 3 ? TY + 2 * EXC + HLO + HHI : 1;
  static constexpr int LV = LZ * LX * LY;
};

// STAGE = false: the fields are gathered from global memory (L2-resident
// tile neighbourhoods) and only the currents live in LDS -- for tiles whose
// staged fields would not fit (3D quadratic shapes).
// The variant that gathers from global memory runs one workgroup per CU (its
// LDS region), two waves per SIMD: it may spend the registers that leaves to
// keep a whole stencil's loads in flight.
// SYP: row stride (nodes) of the 3D LDS current region along y when larger
// than its extent LY, to spread a wave's adds over the LDS banks.
template <typename R, int DIM, int ORDER, int TZ, int TX, int TY, int EXC, int NT, bool DET,
          bool STAGE = true, int SYP = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, STAGE ? 8 : NT / 256))) void
k_gpd_tiled(StepK<R> P, Fields<R> F, PSoA<R> S, TileK T, Ovf<R> O, void* scratch) {
  using TG = TileGeom<DIM, ORDER, TZ, TX, TY, EXC>;
  constexpr int LZ = TG::LZ, LX = TG::LX, LY = TG::LY, LV = TG::LV;
  constexpr int SY = (DIM == 3 && !STAGE && SYP > LY) ? SYP : LY;  // LDS row stride
  constexpr int LVS = LZ * LX * SY;                                  // LDS component stride
  using A = LdsAcc<R, DIM, DET, STAGE>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* sF = reinterpret_cast<R*>(smem_raw);
  // 6 LV sizeof(R) is a multiple of 8
  A* sJ = reinterpret_cast<A*>(STAGE ? (unsigned char*)(sF + 6 * LV) : smem_raw);
  const int t = T.order ? T.order[blockIdx.x] : xcd_remap(blockIdx.x, T.ntiles);
  const int ty = DIM == 3 ? t % T.nty : 0;
  const int tx = (t / T.nty) % T.ntx;
  const int tz = t / (T.nty * T.ntx);
  const int gz0 = T.zc0 + tz * TZ - P.D0.Dint - 1 - EXC - TG::HLO;
  const int gx0 = tx * TX - EXC - TG::HLO;
  const int gy0 = DIM == 3 ? ty * TY - EXC - TG::HLO : 0;
  const Geo& g = P.g;
  // Stage E, B (unconditional loads from a clamped row, zero where the row
  // lies outside the stored grid).  2D: one wave per (component, row), lanes
  // along x, every row of a wave issued before any is stored; the x wrap of a
  // lane and the row offsets are computed once.
  if constexpr (!STAGE) {
  } else if constexpr (DIM == 2) {
    static_assert(LX <= 64, "one wave spans a staged row");
    constexpr int NW = NT / 64, NPAIR = 6 * LZ, PERW = (NPAIR + NW - 1) / NW;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int j = wrap_small(gx0 + (lane < LX ? lane : 0), g.nx);
    R val[PERW];
#pragma unroll
    for (int m = 0; m < PERW; m++) {
      const int q = wv + m * NW;  // (component, row) pair of this wave
      const int qc = q < NPAIR ? q : NPAIR - 1;
      const int comp = qc / LZ, rz = qc - comp * LZ;
      int i = gz0 + rz;
      bool valid = true;
      if (g.periodic_z) i = wrap_small(i, g.nz);
      else {
        valid = i >= -kGuard && i <= g.nz + kGuard;
        i = valid ? i : 0;
      }
      const R x = F.F[comp][(int64_t)(i + kGuard) * g.plane + j];
      val[m] = valid ? x : (R)0;
    }
#pragma unroll
    for (int m = 0; m < PERW; m++) {
      const int q = wv + m * NW;
      if (q < NPAIR && lane < LX) sF[q * LX + lane] = val[m];
    }
  } else {
    constexpr int NST = 6 * LV, PER = 8;
    for (int base = 0; base < NST; base += PER * NT) {
      R val[PER];
#pragma unroll
      for (int m = 0; m < PER; m++) {
        const int v = base + m * NT + (int)threadIdx.x;
        const int vc = v < NST ? v : NST - 1;
        const int comp = vc / LV, rem = vc - comp * LV;
        const int rz = rem / (LX * LY), rxy = rem - rz * (LX * LY);
        const int rx = DIM == 3 ? rxy / LY : rxy;
        int i = gz0 + rz;
        bool valid = true;
        if (g.periodic_z) i = wrap_small(i, g.nz);
        else {
          valid = i >= -kGuard && i <= g.nz + kGuard;
          i = valid ? i : 0;
        }
        const int j = wrap_small(gx0 + rx, g.nx);
        const int k = DIM == 3 ? wrap_small(gy0 + (rxy - rx * LY), g.ny) : 0;
        const R x = F.F[comp][(int64_t)(i + kGuard) * g.plane + (int64_t)j * g.ny + k];
        val[m] = valid ? x : (R)0;
      }
#pragma unroll
      for (int m = 0; m < PER; m++) {
        const int v = base + m * NT + (int)threadIdx.x;
        if (v < NST) sF[v] = val[m];
      }
    }
  }
  for (int v = threadIdx.x; v < 3 * LVS; v += NT) sJ[v] = (A)0;
  // overflow rows reached by far partners, gathered per tile
  __shared__ int far_rows[2];
  // 3D: box of the region's nonzero nodes (first and last node per axis)
  __shared__ int box_lo[3], box_hi[3];
  if (threadIdx.x == 0) {
    far_rows[0] = INT_MAX;
    far_rows[1] = INT_MIN;
    for (int a = 0; a < 3; a++) {
      box_lo[a] = INT_MAX;
      box_hi[a] = INT_MIN;
    }
  }
  __syncthreads();
  LdsSinkT<A, LX, SY, DET> ls{sJ, LVS};
  const int p0 = T.start[t], p1 = T.start[t + 1];
  // 3D: this thread's box of the region nodes its particles deposit to
  int blo[3] = {INT_MAX, INT_MAX, INT_MAX}, bhi[3] = {INT_MIN, INT_MIN, INT_MIN};
  auto particles = [&](const auto& lf) {
    // the whole state of the next particle is loaded while this one is pushed
    int p = p0 + (int)threadIdx.x;
    int id_n = -1;
    R xn[3] = {(R)0, (R)0, (R)0}, un[3] = {(R)0, (R)0, (R)0}, wn = (R)0;
    if (p < p1) {
      id_n = S.id[p];
      load_state(S, p, xn, un, wn);
    }
    for (; p < p1; p += NT) {
      const int id = id_n;
      R xi[3] = {xn[0], xn[1], xn[2]}, du[3] = {un[0], un[1], un[2]};
      const R w = wn;
      if (p + NT < p1) {
        id_n = S.id[p + NT];
        load_state(S, p + NT, xn, un, wn);
      }
      if (id < 0) continue;
      Birth b = decode_id(P.L, id);
      R r[3];
      birth_offsets<R, DIM>(P.L, id, r);
      Pos<R> i0 = ion_at<R, DIM>(b, r, P.D0);
      Pos<R> e0 = add_xi<R, DIM>(i0, xi);
      // cells relative to the LDS region (wrapped where the axis is periodic)
      int rz = e0.c[0] - gz0, riz = i0.c[0] - gz0;
      if (g.periodic_z) {
        rz = wrap_once(rz, g.nz);
        riz = wrap_once(riz, g.nz);
      }
      const int rx = wrap_once(e0.c[1] - gx0, g.nx), rix = wrap_once(i0.c[1] - gx0, g.nx);
      // the electron's stencil must lie in the region; the partner's may not
      // (its separate stencil then reaches the overflow grid)
      bool inside = rz >= TG::HLO && rz < LZ - TG::HHI && rx >= TG::HLO && rx < LX - TG::HHI;
      bool near = riz >= TG::HLO && riz < LZ - TG::HHI && rix >= TG::HLO && rix < LX - TG::HHI;
      int ry = 0;
      if (DIM == 3) {
        ry = wrap_once(e0.c[2] - gy0, g.ny);
        const int riy = wrap_once(i0.c[2] - gy0, g.ny);
        inside = inside && ry >= TG::HLO && ry < LY - TG::HHI;
        near = near && riy >= TG::HLO && riy < LY - TG::HHI;
      }
      if (!inside) {
        T.strag[atomicAdd(T.nstrag, 1)] = p;
        continue;
      }
      Pos<R> i1 = ion_at<R, DIM>(b, r, P.D1);
      int bc[3] = {rz, rx, ry};
      bool dead = particle_step<R, DIM, ORDER>(P, lf, ls, bc, e0, i0, i1, xi, du, w, NoHook(), near);
      if constexpr (DIM == 3) {
        // Per axis the deposit's nonzero values lie on the nodes from the
        // lower to the higher of the old and new shape bases plus ORDER (the
        // window's last node, one past the shapes, takes only zeros when the
        // base does not change), at region index bc + (node - e0.c); the
        // partner's nodes too when it deposits here.
        const Pos<R> e1 = add_xi<R, DIM>(i1, xi);
#pragma unroll
        for (int a = 0; a < 3; a++) {
          const int s = bc[a] - e0.c[a];
          const int b0 = shape_base<R, ORDER>(e0.c[a], e0.o[a]);
          const int b1 = shape_base<R, ORDER>(e1.c[a], e1.o[a]);
          int lo = min(b0, b1), hi = max(b0, b1);
          if (near) {
            const int c0 = shape_base<R, ORDER>(i0.c[a], i0.o[a]);
            const int c1 = shape_base<R, ORDER>(i1.c[a], i1.o[a]);
            lo = min(lo, min(c0, c1));
            hi = max(hi, max(c0, c1));
          }
          blo[a] = min(blo[a], lo + s);
          bhi[a] = max(bhi[a], hi + ORDER + s);
        }
      }
      if (!near) {
        atomicMin(&far_rows[0], min(e0.c[0], i0.c[0]) - ORDER - 1);
        atomicMax(&far_rows[1], max(e0.c[0], i0.c[0]) + ORDER + 2);
        partner_far<R, DIM, ORDER, DET>(P, O, i0, i1, w);
      }
      store_state<R, DIM>(S, p, xi, du, dead);
    }
  };
  if constexpr (STAGE) {
    particles(LdsFetch<R, LX, LY>{sF, LV});
  } else {
    const int gzr = g.periodic_z ? wrapi(gz0, g.nz) : gz0;
    // a region inside the grid along y: the stencils' y rows load as vectors
    if (DIM == 3 && gy0 >= 0 && gy0 + LY <= g.ny)
      particles(RegionFetch<R, true>{(const R* const*)F.F, g, gzr, gx0, gy0});
    else
      particles(RegionFetch<R>{(const R* const*)F.F, g, gzr, gx0, gy0});
  }
  __syncthreads();
  if (threadIdx.x == 0 && far_rows[0] <= far_rows[1]) {
    atomicMin(&O.rows[0], g.periodic_z ? 0 : far_rows[0]);
    atomicMax(&O.rows[1], g.periodic_z ? g.nz : far_rows[1]);
  }
  using D = typename std::conditional<DET, long long, R>::type;
  D* dst = reinterpret_cast<D*>(scratch) + (int64_t)t * 3 * LV;
  if constexpr (DIM == 3) {
    // Only the box of the nodes the particles deposited to is stored
    // (outside it every node of the region is zero), which cuts the flush
    // and the fold's reads to what the tile's particles reached.
    static_assert(LZ < 32 && LX < 32 && LY < 32, "box fields of 5 bits");
    static_assert(3 * LV < (1 << 14), "exact FP32 index division");
#pragma unroll
    for (int a = 0; a < 3; a++) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        blo[a] = min(blo[a], __shfl_xor(blo[a], o));
        bhi[a] = max(bhi[a], __shfl_xor(bhi[a], o));
      }
    }
    if ((threadIdx.x & 63) == 0 && bhi[0] != INT_MIN) {
      for (int a = 0; a < 3; a++) {
        atomicMin(&box_lo[a], blo[a]);
        atomicMax(&box_hi[a], bhi[a]);
      }
    }
    __syncthreads();
    // clipped to the region (every deposit lies inside it)
    const int z0 = max(box_lo[0], 0), x0 = max(box_lo[1], 0), y0 = max(box_lo[2], 0);
    const int z1 = min(box_hi[0], LZ - 1), x1 = min(box_hi[1], LX - 1), y1 = min(box_hi[2], LY - 1);
    const bool any = z0 <= z1 && x0 <= x1 && y0 <= y1;
    const int nz = any ? z1 - z0 + 1 : 0, nx = any ? x1 - x0 + 1 : 0, ny = any ? y1 - y0 + 1 : 0;
    const int nxy = nx * ny, vol = nz * nxy;
    // u / n as floor((u + 1/2) (1/n)) in FP32: exact for u below 2^14 (the
    // fraction of (u + 1/2) / n stays 1/(2n) away from an integer, far above
    // the rounding of the product)
    const float rvol = 1.0f / (float)max(vol, 1), rxy = 1.0f / (float)max(nxy, 1),
                rny = 1.0f / (float)max(ny, 1);
    for (int u = threadIdx.x; u < 3 * vol; u += NT) {
      const int c = (int)(((float)u + 0.5f) * rvol);
      const int e = u - c * vol;
      const int z = (int)(((float)e + 0.5f) * rxy);
      const int f = e - z * nxy;
      const int x = (int)(((float)f + 0.5f) * rny);
      const int y = f - x * ny;
      dst[u] = (D)sJ[c * LVS + ((z0 + z) * LX + (x0 + x)) * SY + (y0 + y)];
    }
    if (threadIdx.x == 0) T.box[t] = any ? pack_box(z0, nz, x0, nx, y0, ny) : 0u;
  } else {
    static_assert(SY == LY, "padded rows in 3D only");
    for (int v = threadIdx.x; v < 3 * LV; v += NT) dst[v] = (D)sJ[v];
  }
}

// --------------------------------------------------------------------------
// Plasma creation: lattice columns [k0, k0 + ncols) -> slots starting at
// counts[0] (the current slot count); each slot gets id, xi = 0, du = du0
// and the weight gamma_b n_lab(z_lab) c(x, y) dV / ppc at z_lab = gamma_b (k + r_z) dz,
// with c the plasma channel's transverse factor.
// --------------------------------------------------------------------------
struct DensityK {
  double n_uniform;
  int nknots;
  double kz[32], kn[32];
  double gamma_b, dz, dV_over_ppc;
  double du0[3];
  // channel: 1 + ch_k ((x dx - xa)^2 + (y dy - ya)^2), ch_k = depth / radius^2
  double ch_k, dx, dy, xa, ya;
  int dim3;
};

// Transverse factor of the plasma channel at the birth position (cells).
__device__ __forceinline__ double channel_factor(const DensityK& d, double x, double y) {
  if (d.ch_k == 0.0) return 1.0;
  const double a = x * d.dx - d.xa;
  const double b = d.dim3 ? y * d.dy - d.ya : 0.0;
  return 1.0 + d.ch_k * (a * a + b * b);
}

// Channel factor of a lattice birth.
__device__ __forceinline__ double birth_channel(const DensityK& d, const LatticeP& L, int id,
                                                const Birth& b) {
  if (d.ch_k == 0.0) return 1.0;
  const double x = (double)b.j + (double)birth_offset<double>(L, id, 1);
  const double y = d.dim3 ? (double)b.l + (double)birth_offset<double>(L, id, 2) : 0.0;
  return channel_factor(d, x, y);
}

__device__ __forceinline__ double lab_density(const DensityK& d, double zl) {
  if (d.nknots < 2) return d.n_uniform;
  if (zl < d.kz[0] || zl > d.kz[d.nknots - 1]) return 0.0;
  for (int m = 0; m + 1 < d.nknots; m++) {
    if (zl <= d.kz[m + 1]) {
      double f = (zl - d.kz[m]) / (d.kz[m + 1] - d.kz[m]);
      return d.kn[m] + f * (d.kn[m + 1] - d.kn[m]);
    }
  }
  return d.kn[d.nknots - 1];
}

template <typename R>
__global__ __launch_bounds__(256) void k_create(PSoA<R> S, LatticeP L, DensityK d, int k0,
                                                int64_t count, const int* counts) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const int base = counts[0];
  int id = (int)((int64_t)k0 * L.nyy * L.nx * L.ppc + q);
  int p = base + (int)q;
  Birth b = decode_id(L, id);
  double rz = (double)birth_offset<double>(L, id, 0);
  double zl = d.gamma_b * ((double)b.k + rz) * d.dz;
  double w = d.gamma_b * lab_density(d, zl) * birth_channel(d, L, id, b) * d.dV_over_ppc;
  S.id[p] = id;
  S.xi[0][p] = (R)0;
  S.xi[1][p] = (R)0;
  if (S.xi[2]) S.xi[2][p] = (R)0;
  S.du[0][p] = (R)d.du0[0];
  S.du[1][p] = (R)d.du0[1];
  S.du[2][p] = (R)d.du0[2];
  S.w[p] = (R)w;
}

__global__ void k_bump_slots(int* counts, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counts[0] += add;
}

// Export of every slot as absolute FP64 state (electron position in grid
// cells relative to the window; momentum u = du + u_b z).
template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_export(PSoA<R> S, LatticeP L, Drift<R> D, double ub,
                                                const int* counts, double* z, double* x,
                                                double* y, double* ux, double* uy, double* uz,
                                                double* w, int* ido) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= counts[0]) return;
  int id = S.id[p];
  ido[p] = id;
  if (id < 0) return;
  R xi[3], du[3], ww;
  load_state(S, p, xi, du, ww);
  Birth b = decode_id(L, id);
  Pos<R> e = add_xi<R, DIM>(ion_pos<R, DIM>(L, id, b, D), xi);
  z[p] = (double)e.c[0] + (double)e.o[0];
  x[p] = (double)e.c[1] + (double)e.o[1];
  y[p] = DIM == 3 ? (double)e.c[2] + (double)e.o[2] : 0.0;
  ux[p] = (double)du[0];
  uy[p] = (double)du[1];
  uz[p] = ub + (double)du[2];
  w[p] = (double)ww;
}

}  // namespace bfpic
