// device_common.hpp -- shared device-side definitions of the boosted-frame PIC
// library: grid geometry and indexing, the counter-based generator, particle
// position reconstruction, shape factors and the split-form Boris push.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bfpic {

constexpr int kGuard = 6;  // stored rows beyond each z end of the domain

// Grid geometry.  Component arrays are [row][j][k] with row = i + kGuard,
// i in [-kGuard, nz + kGuard]; k (y) fastest; ny = 1 in 2D.
struct Geo {
  int nz, nx, ny;
  int periodic_z;
  int64_t plane;  // nx * ny
  int64_t rows;   // nz + 2 kGuard + 1
};

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Wrap into [0, n) for x in (-n, 2n); other values take the full modulo.
__device__ __forceinline__ int wrap_small(int x, int n) {
  if (x < 0) x += n;
  else if (x >= n) x -= n;
  if ((unsigned)x >= (unsigned)n) x = wrapi(x, n);
  return x;
}

// Storage index of node (i, j, k) or -1 outside storage (open z only).  Node
// indices lie within a few cells of the grid, where one period of wrap is
// exact; farther ones take the modulo.
__device__ __forceinline__ int64_t gidx(const Geo& g, int i, int j, int k) {
  if (g.periodic_z) i = wrap_small(i, g.nz);
  else if (i < -kGuard || i > g.nz + kGuard) return -1;
  j = wrap_small(j, g.nx);
  k = g.ny > 1 ? wrap_small(k, g.ny) : 0;
  return ((int64_t)(i + kGuard) * g.nx + j) * g.ny + k;
}

// Domain rows of a component: integer-z components own rows [0, nz] (both
// boundary planes), half-z components [0, nz - 1]; periodic: [0, nz - 1].
__device__ __forceinline__ int row_hi(const Geo& g, int half_z) {
  return (g.periodic_z || half_z) ? g.nz - 1 : g.nz;
}
__device__ __forceinline__ bool in_domain(const Geo& g, int half_z, int i) {
  return i >= 0 && i <= row_hi(g, half_z);
}

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood 2014): output n of the generator started at
// state `seed`.  In-cell offsets take its top 24 bits times 2^-24, exact in
// both float and double.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t n) {
  uint64_t z = seed + n * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Division by a runtime-invariant divisor d >= 1 for 0 <= n < 2^31
// (Granlund & Montgomery 1994): l = ceil(log2 d), m = 2^32 (2^l - d) / d + 1,
// n / d = (umulhi(m, n) + n) >> l.  The host fills (m, l); d = 1 has m = l = 0.
struct FastDiv {
  uint32_t m;
  int l;
  int d;
};

__device__ __forceinline__ int fdiv(const FastDiv& f, int n) {
  uint32_t t = __umulhi(f.m, (uint32_t)n);
  return (int)((t + (uint32_t)n) >> f.l);
}

// Particle identity: id = ((k * nyy + l) * nx + j) * ppc + s for lattice
// column k, transverse cells (j, l) and slot s.  The generator counter of
// axis a (0 z, 1 x, 2 y) is 4 id + a + 1.
struct Birth {
  int k, j, l;
};

struct LatticeP {
  uint64_t seed;
  int ppc, nx, nyy;
  int load;  // 0 random, 1 centred
  FastDiv dppc, dnx, dnyy;
};

__device__ __forceinline__ Birth decode_id(const LatticeP& L, int id) {
  Birth b;
  int q = fdiv(L.dppc, id);
  int r = fdiv(L.dnx, q);
  b.j = q - r * L.nx;
  int t = fdiv(L.dnyy, r);
  b.l = r - t * L.nyy;
  b.k = t;
  return b;
}

// One period of wrap, without branches: exact for x in [-n, 2n); callers that
// test the result against a range inside [0, n) reject anything else.
__device__ __forceinline__ int wrap_once(int x, int n) {
  return x + (x < 0 ? n : 0) - (x >= n ? n : 0);
}

// In-cell birth offsets: 24-bit fields of SplitMix64 outputs times 2^-24
// (exact in FP32 and FP64).  Output 2 id + 1 gives z (bits 63..40) and x
// (bits 39..16); output 2 id + 2 gives y (bits 63..40).
__device__ __forceinline__ uint64_t birth_bits(const LatticeP& L, int id, int second) {
  return splitmix64(L.seed, 2ULL * (uint64_t)id + 1ULL + (uint64_t)second);
}

// Fields are taken from 32-bit halves (a 64-bit integer costs more to convert).
template <typename R>
__device__ __forceinline__ R offset_hi(uint64_t r) {
  return (R)((uint32_t)(r >> 32) >> 8) * (R)(1.0 / 16777216.0);
}
template <typename R>
__device__ __forceinline__ R offset_mid(uint64_t r) {
  return (R)(((uint32_t)r >> 16) | (((uint32_t)(r >> 32) & 0xFFu) << 16)) *
         (R)(1.0 / 16777216.0);
}

template <typename R>
__device__ __forceinline__ R birth_offset(const LatticeP& L, int id, int axis) {
  if (L.load) return (R)0.5;
  const uint64_t r = birth_bits(L, id, axis == 2);
  return axis == 1 ? offset_mid<R>(r) : offset_hi<R>(r);
}

// A particle position as an integer cell plus an offset in [0, 1).
template <typename R>
struct Pos {
  int c[3];
  R o[3];
};

// Renormalise cell + off (off may leave [0,1)).  If the offset rounds to 1
// after the subtraction, move to the next cell with offset 0.
template <typename R>
__device__ __forceinline__ void renorm(int& c, R& o) {
  R f = floor(o);
  c += (int)f;
  o -= f;
  if (o >= (R)1) {
    c += 1;
    o = (R)0;
  }
}

// Drift of the rigid ion lattice at a step: D = Dint + Dfrac, Dfrac in [0,1),
// in cells along z (plasma drift n beta_b dt / dz plus window displacement).
template <typename R>
struct Drift {
  int Dint;
  R Dfrac;
};

// Ion partner position from its birth cell and in-cell offsets r: the birth
// spot minus the drift (x, y never move).
template <typename R, int DIM>
__device__ __forceinline__ Pos<R> ion_at(const Birth& b, const R r[3], const Drift<R>& D) {
  Pos<R> p;
  p.c[0] = b.k - D.Dint;
  p.o[0] = r[0] - D.Dfrac;  // exact in FP32: both are multiples of 2^-24
  if (p.o[0] < (R)0) {
    p.o[0] += (R)1;
    p.c[0] -= 1;
  }
  p.c[1] = b.j;
  p.o[1] = r[1];
  p.c[2] = DIM == 3 ? b.l : 0;
  p.o[2] = DIM == 3 ? r[2] : (R)0;
  return p;
}

template <typename R, int DIM>
__device__ __forceinline__ void birth_offsets(const LatticeP& L, int id, R r[3]) {
  if (L.load) {
    r[0] = r[1] = (R)0.5;
    r[2] = DIM == 3 ? (R)0.5 : (R)0;
    return;
  }
  const uint64_t a = birth_bits(L, id, 0);
  r[0] = offset_hi<R>(a);
  r[1] = offset_mid<R>(a);
  r[2] = DIM == 3 ? offset_hi<R>(birth_bits(L, id, 1)) : (R)0;
}

template <typename R, int DIM>
__device__ __forceinline__ Pos<R> ion_pos(const LatticeP& L, int id, const Birth& b,
                                          const Drift<R>& D) {
  R r[3];
  birth_offsets<R, DIM>(L, id, r);
  return ion_at<R, DIM>(b, r, D);
}

// Electron position = ion partner + peculiar displacement xi (cells).
template <typename R, int DIM>
__device__ __forceinline__ Pos<R> add_xi(Pos<R> p, const R xi[3]) {
#pragma unroll
  for (int a = 0; a < DIM; a++) {
    p.o[a] += xi[a];
    renorm(p.c[a], p.o[a]);
  }
  return p;
}

// ---------------------------------------------------------------------------
// Shape factors of order 1 (linear) and 2 (quadratic B-spline).  For a
// position cell c + offset o, on the integer lattice (half = 0) or the
// half-integer lattice (half = 1, node index m sits at m + 1/2), return the
// first node b and weights w[0..ORDER] of nodes b..b+ORDER.
// ---------------------------------------------------------------------------
template <typename R, int ORDER>
__device__ __forceinline__ int shape(int c, R o, int half, R w[ORDER + 1]) {
  if (ORDER == 1) {
    int b = c;
    R f = o;
    if (half) {
      if (o >= (R)0.5) f = o - (R)0.5;
      else {
        b = c - 1;
        f = o + (R)0.5;
      }
    }
    w[0] = (R)1 - f;
    w[1] = f;
    return b;
  } else {
    int m;
    R d;
    if (half) {
      m = c;
      d = o - (R)0.5;
    } else if (o >= (R)0.5) {
      m = c + 1;
      d = o - (R)1;
    } else {
      m = c;
      d = o;
    }
    R a = (R)0.5 - d, e = (R)0.5 + d;
    w[0] = (R)0.5 * a * a;
    w[1] = (R)0.75 - d * d;
    w[ORDER] = (R)0.5 * e * e;
    return m - 1;
  }
}

// First node of shape(c, o, 0, w) on the integer lattice, without the weights.
template <typename R, int ORDER>
__device__ __forceinline__ int shape_base(int c, R o) {
  if (ORDER == 1) return c;
  return o >= (R)0.5 ? c : c - 1;
}

// Energy-conserving (Galerkin) gather: on the half-integer lattice the shape
// of one order lower, written on the node window of shape(c, o, 1, w) so that
// it reads the same nodes: order 0 (the half node c + 1/2 of the particle's
// cell) for ORDER 1, linear on the half nodes for ORDER 2.
template <typename R, int ORDER>
__device__ __forceinline__ void shape_half_reduced(R o, R w[ORDER + 1]) {
  const bool hi = o >= (R)0.5;
  if (ORDER == 1) {
    // window (c - 1, c) for o < 1/2, (c, c + 1) for o >= 1/2
    w[0] = hi ? (R)1 : (R)0;
    w[1] = hi ? (R)0 : (R)1;
  } else {
    // window (c - 1, c, c + 1); the linear pair is (c, c + 1) for o >= 1/2,
    // (c - 1, c) below
    const R f = hi ? o - (R)0.5 : o + (R)0.5;
    w[0] = hi ? (R)0 : (R)1 - f;
    w[1] = hi ? (R)1 - f : f;
    w[ORDER] = hi ? f : (R)0;
  }
}

// ---------------------------------------------------------------------------
// Relativistic Boris push (Boris 1970) on the peculiar momentum du = u - ub z,
// written so that no step subtracts two numbers of size gamma_b:
//   gamma^2 = gb^2 + c,  c = 2 ub du_z + |du|^2,  gamma - gb = c / (gb + gamma)
//   rotation terms (ub + du_z) t split into ub t + du_z t
//   v_z - v_b = ((2 + gb (gamma - gb)) du_z - ub |du|^2) / ((gamma + gb) gamma gb)
// ub, gb: drift momentum and its gamma (gb^2 = 1 + ub^2 in FP64, rounded once).
// ---------------------------------------------------------------------------
template <typename R>
struct PushC {
  R ub, gb, gb2;  // drift
  R qdt2;         // q dt / 2 (q = -1)
};

// Reciprocal: the hardware estimate (1 ulp) in FP32, exact division in FP64.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

// Square root: the hardware instruction (1 ulp) in FP32, correctly rounded in FP64.
__device__ __forceinline__ float root(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double root(double x) { return sqrt(x); }

template <typename R>
__device__ __forceinline__ R gamma_minus_gb(const PushC<R>& P, R dux, R duy, R duz) {
  R c = (R)2 * P.ub * duz + (dux * dux + duy * duy + duz * duz);
  return c * rcp(P.gb + root(P.gb2 + c));
}

template <typename R>
__device__ __forceinline__ void boris_split(const PushC<R>& P, const R E[3], const R B[3],
                                            R du[3], R dv[3], R& gam) {
  // vectors in (x, y, z) order
  R mx = du[0] + P.qdt2 * E[0];
  R my = du[1] + P.qdt2 * E[1];
  R mz = du[2] + P.qdt2 * E[2];
  R g = P.gb + gamma_minus_gb(P, mx, my, mz);
  R f = P.qdt2 * rcp(g);
  R tx = f * B[0], ty = f * B[1], tz = f * B[2];
  R sfac = (R)2 * rcp((R)1 + (tx * tx + ty * ty + tz * tz));
  // u' = u- + u- x t, with u-_z = ub + mz
  R px = mx + (my * tz - (P.ub * ty + mz * ty));
  R py = my + ((P.ub * tx + mz * tx) - mx * tz);
  R pz = mz + (mx * ty - my * tx);
  R sx = sfac * tx, sy = sfac * ty, sz = sfac * tz;
  // u+ = u- + u' x s, with u'_z = ub + pz
  R qx = mx + (py * sz - (P.ub * sy + pz * sy));
  R qy = my + ((P.ub * sx + pz * sx) - px * sz);
  R qz = mz + (px * sy - py * sx);
  du[0] = qx + P.qdt2 * E[0];
  du[1] = qy + P.qdt2 * E[1];
  du[2] = qz + P.qdt2 * E[2];
  R dg = gamma_minus_gb(P, du[0], du[1], du[2]);
  gam = P.gb + dg;
  R ig = rcp(gam);
  dv[0] = du[0] * ig;
  dv[1] = du[1] * ig;
  R u2 = du[0] * du[0] + du[1] * du[1] + du[2] * du[2];
  dv[2] = (((R)2 + P.gb * dg) * du[2] - P.ub * u2) * (ig * rcp((gam + P.gb) * P.gb));
}

// XCD-aware block -> work item map: consecutive work items land on the same
// XCD (blocks are dealt round-robin over the 8 XCDs), so neighbouring tiles
// share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int X = 8;
  int per = n / X, rem = n % X;
  int x = b % X, idx = b / X;
  return x < rem ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

// Box of a 3D tile region's nonzero nodes, one word per tile: first node
// and extent along z, x, y, 5 bits each (regions are under 32 nodes per
// axis).  A zero word is the empty box.  The region's scratch slot holds
// just the box, component-major, z-major within a component.
struct RegionBox {
  int z0, nz, x0, nx, y0, ny;
  __device__ __forceinline__ int vol() const { return nz * nx * ny; }
};
__device__ __forceinline__ unsigned pack_box(int z0, int nz, int x0, int nx, int y0, int ny) {
  return (unsigned)z0 | ((unsigned)nz << 5) | ((unsigned)x0 << 10) | ((unsigned)nx << 15) |
         ((unsigned)y0 << 20) | ((unsigned)ny << 25);
}
__device__ __forceinline__ RegionBox unpack_box(unsigned w) {
  RegionBox b;
  b.z0 = (int)(w & 31u);
  b.nz = (int)((w >> 5) & 31u);
  b.x0 = (int)((w >> 10) & 31u);
  b.nx = (int)((w >> 15) & 31u);
  b.y0 = (int)((w >> 20) & 31u);
  b.ny = (int)((w >> 25) & 31u);
  return b;
}

}  // namespace bfpic
