// kernels_fields.hpp -- current fold + binomial filter, Yee update with Mur
// boundaries, window shift, boosted laser initialisation, field copies.
#pragma once

#include <type_traits>

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
  const void* scratch;  // [tile][3][LV] of R, or of int64 in deterministic mode
  double inv_scale;     // deterministic mode: value of one fixed-point unit
  int ntz, ntx, nty, ntiles;
  int gz0, gx0, gy0;  // region origin of tile (0,0,0) in grid cells
  int TZ, TX, TY, LZ, LX, LY, LV;
  int64_t zero_base;    // element offset of the row of zero tiles past the last tile
  const unsigned* box;  // 3D: per tile, the box of its region's nonzero nodes (the
                        // slot holds just the box)
  Ovf<R> o;
};

// Candidate tiles of a node along one axis: the regions are spaced T apart
// and are L <= 3 T long, so node offset q (from the region origin of tile 0)
// lies in tile h = q / T at local q - h T, and in tiles h - 1, h - 2 at local
// q - h T + T, + 2 T when that is below L.
template <typename R, int DIM, int TZ, int TX, int TY, bool DET>
__device__ __forceinline__ R fold_at(const FoldK<R>& K, const Geo& g, int comp, int i, int j,
                                     int k) {
  using A = typename std::conditional<DET, long long, R>::type;
  const A* scratch = reinterpret_cast<const A*>(K.scratch);
  A acc = (A)0;
  if (g.periodic_z) i = wrap_small(i, g.nz);  // halo rows of the filter may lie beyond the seam
  if (K.ntiles > 0) {
    int qz = i - K.gz0;
    if (g.periodic_z) qz = wrap_small(qz, g.nz);
    const int qx = wrap_small(j - K.gx0, g.nx);
    const int qy = DIM == 3 ? wrap_small(k - K.gy0, g.ny) : 0;
    const int hz = qz >= 0 ? qz / TZ : -((TZ - 1 - qz) / TZ);
    const int hx = qx / TX, hy = DIM == 3 ? qy / TY : 0;
    const int lz = qz - hz * TZ, lx = qx - hx * TX, ly = qy - hy * TY;
    // Every candidate is loaded unconditionally, so that all the loads of a
    // node are in flight together: a tile that does not cover the node reads
    // the zeroed tile row kept past the last tile.
#pragma unroll
    for (int a = 0; a < 3; a++) {
      int tz = hz - a;
      const int rz = lz + a * TZ;
      if (g.periodic_z && tz < 0) tz += K.ntz;
      const bool vz = tz >= 0 && tz < K.ntz && rz < K.LZ;
#pragma unroll
      for (int b = 0; b < 3; b++) {
        int tx = hx - b;
        const int rx = lx + b * TX;
        if (tx < 0) tx += K.ntx;
        const bool vx = vz && rx < K.LX;
#pragma unroll
        for (int c = 0; c < (DIM == 3 ? 3 : 1); c++) {
          int ty = hy - c;
          const int ry = ly + c * TY;
          if (ty < 0) ty += K.nty;
          const bool v = vx && (DIM != 3 || ry < K.LY);
          const int t = (tz * K.ntx + tx) * K.nty + ty;
          int64_t e = K.zero_base;
          if constexpr (DIM == 3) {
            const unsigned w = K.box[v ? t : 0];
            const RegionBox bx = unpack_box(v ? w : 0u);
            const int oz = rz - bx.z0, ox = rx - bx.x0, oy = ry - bx.y0;
            if ((unsigned)oz < (unsigned)bx.nz && (unsigned)ox < (unsigned)bx.nx &&
                (unsigned)oy < (unsigned)bx.ny)
              e = (int64_t)t * 3 * K.LV + comp * bx.vol() + (oz * bx.nx + ox) * bx.ny + oy;
          } else {
            if (v) e = ((int64_t)t * 3 + comp) * K.LV + (rz * K.LX + rx) * K.LY + ry;
          }
          acc += scratch[e];
        }
      }
    }
  }
  int r0 = K.o.rows[0], r1 = K.o.rows[1];
  if (i >= r0 && i <= r1) {
    int64_t n = gidx(g, i, j, k);
    if constexpr (DET) {
      if (n >= 0) acc += K.o.Jq[comp][n];
    } else {
      if (n >= 0) acc += K.o.J[comp][n];
    }
  }
  if constexpr (DET) return (R)((double)acc * K.inv_scale);
  else return acc;
}

// Filter: per axis N passes of (1/4, 1/2, 1/4) then (-N/4, 1 + N/2, -N/4)
// when compensating; outside an open z domain the current counts as zero.
// One workgroup filters an FZ x FX [x FY] output tile of one component with
// a halo of H = N (+1) nodes, all passes in LDS.  Work is laid out as rows
// (one wave each) by lanes along the contiguous axis (x in 2D, y in 3D).
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
  const int LN = DIM == 3 ? NY : NX;       // lane axis length
  const int NR = DIM == 3 ? NZ * NX : NZ;  // rows
  const int NV = NR * LN;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  R* A = lds;
  R* Bq = lds + NV;
  for (int row = wv; row < NR; row += nw) {
    const int rz = DIM == 3 ? row / NX : row;
    const int rx = DIM == 3 ? row - rz * NX : 0;
    const int i = i0 - H + rz;
    const bool ok = g.periodic_z || in_domain(g, half_z, i);
    for (int c = lane; c < LN; c += 64) {
      const int j = DIM == 3 ? j0 - H + rx : j0 - H + c;
      const int k = DIM == 3 ? k0 - H + c : 0;
      A[row * LN + c] = ok ? src(i, j, k) : (R)0;
    }
  }
  __syncthreads();
  const int naxes = DIM == 3 ? 3 : 2;
  const int npass = fk.passes + (fk.comp && fk.passes > 0 ? 1 : 0);
  for (int axis = 0; axis < naxes; axis++) {
    // neighbour stride in A and the length of the axis
    const int stride = axis == 0 ? (DIM == 3 ? NX * NY : NX) : (axis == 1 && DIM == 3 ? NY : 1);
    const int len = axis == 0 ? NZ : (axis == 1 ? NX : NY);
    for (int p = 0; p < npass; p++) {
      const R a = p < fk.passes ? (R)0.25 : (R)fk.a_c;
      const R b = p < fk.passes ? (R)0.5 : (R)fk.b_c;
      for (int row = wv; row < NR; row += nw) {
        const int rz = DIM == 3 ? row / NX : row;
        const int rx = DIM == 3 ? row - rz * NX : 0;
        const bool zero_row = axis == 0 && !g.periodic_z && !in_domain(g, half_z, i0 - H + rz);
        for (int c = lane; c < LN; c += 64) {
          const int v = row * LN + c;
          const int pos = axis == 0 ? rz : (axis == 1 ? (DIM == 3 ? rx : c) : c);
          R val = (pos == 0 || pos == len - 1) ? A[v]
                                               : a * A[v - stride] + b * A[v] + a * A[v + stride];
          Bq[v] = zero_row ? (R)0 : val;
        }
      }
      __syncthreads();
      R* t = A;
      A = Bq;
      Bq = t;
    }
  }
  const int fy = DIM == 3 ? FY : 1;
  const int ORW = DIM == 3 ? FZ * FX : FZ;  // output rows
  const int OLN = DIM == 3 ? fy : FX;
  for (int row = wv; row < ORW; row += nw) {
    const int r = DIM == 3 ? row / FX : row;
    const int s = DIM == 3 ? row - r * FX : 0;
    const int i = i0 + r;
    if (!in_domain(g, half_z, i)) continue;
    for (int c = lane; c < OLN; c += 64) {
      const int j = DIM == 3 ? j0 + s : j0 + c;
      const int k = DIM == 3 ? k0 + c : 0;
      if (j >= g.nx || (DIM == 3 && k >= g.ny)) continue;
      const int v = DIM == 3 ? ((r + H) * NX + (s + H)) * NY + (c + H) : (r + H) * NX + (c + H);
      out[gidx(g, i, j, k)] = A[v];
    }
  }
  __syncthreads();
}

template <typename R, int DIM, int TZ, int TX, int TY, bool DET>
struct FoldSrc {
  const FoldK<R>* K;
  Geo g;
  int comp;
  __device__ __forceinline__ R operator()(int i, int j, int k) const {
    return fold_at<R, DIM, TZ, TX, TY, DET>(*K, g, comp, i, j, k);
  }
};

template <typename R, int DIM, int FZ, int FX, int FY, int TZ, int TX, int TY, bool DET>
__global__ __launch_bounds__(256) void k_fold_filter(Geo g, FoldK<R> K, FiltK fk, Fields<R> Jf,
                                                     int nbz, int nbx, int nby) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* lds = reinterpret_cast<R*>(smem_raw);
  int nb = nbz * nbx * nby;
  int b = xcd_remap(blockIdx.x, nb);
  int by = b % nby, bx = (b / nby) % nbx, bz = b / (nby * nbx);
  int i0 = bz * FZ, j0 = bx * FX, k0 = by * FY;
  for (int comp = 0; comp < 3; comp++) {
    FoldSrc<R, DIM, TZ, TX, TY, DET> src{&K, g, comp};
    filter_tile<R, DIM, FZ, FX, FY>(g, fk, half_z_j(comp), i0, j0, k0, src, Jf.F[comp], lds);
  }
}

// 2D fold + filter on register columns.  A wave owns NC of the three current
// components (1 or 3; blockIdx.y picks them) over a window of WT TZ output
// rows (the z extent of WT rows of co-moving tiles, so that every row's
// candidate tiles and local row are fixed at compile time; the 2 NP halo rows
// are read once per window, so longer windows re-read less) by 64 - 2 NP
// output columns.  Lane c holds column j0 - NP + c over the TZ + 2 NP rows
// the filter needs; the z passes run in registers, the x passes exchange
// neighbours across lanes.  After NP passes along an axis the values NP or
// more nodes inside the window are exact; those are stored.  Tile rows
// outside the co-moving range read a row of zero tiles kept past the last
// tile, so every load is unconditional.  No LDS and no barriers.
//
// The fold sums, per node, the tile whose core holds it, then the tile
// before it in z, each with the two x candidates, then the overflow grid:
// the order of fold_at.
// A wave that folds all three components gets the register budget of four
// waves per SIMD, so that each window's loads are all in flight at once.
template <typename R, int NP, int TZ, int TX, int LZ, int LX, bool DET, int NC, int WT = 1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, NC == 3 ? 4 : 8))) void
k_fold_filter_cols(Geo g, FoldK<R> K, FiltK fk, Fields<R> Jf, int tz_lo, int nseg, int nbx,
                   int zero_row) {
  constexpr int H = NP, L = WT * TZ + 2 * H;
  constexpr int FX = 64 - 2 * H;
  static_assert(H <= TZ && LZ <= 2 * TZ, "window geometry");
  const int lane = threadIdx.x & 63;
  // the window index is the same for the whole wave: keep it (and the row
  // arithmetic derived from it) in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * 4 +
                                               (int)(threadIdx.x >> 6));
  if (w >= nseg * nbx) return;  // the whole wave leaves together
  const int sw = w / nbx, bx = w - sw * nbx;
  const int tzw = tz_lo + sw * WT;
  const int iw0 = K.gz0 + tzw * TZ;  // first output row of the window
  const int j0 = bx * FX;
  const int j = j0 - H + lane;
  const bool out_lane = lane >= H && lane < 64 - H && j < g.nx;
  const int jl = lane == 0 ? 63 : lane - 1, jr = lane == 63 ? 0 : lane + 1;
  // x candidates of this lane's column: tile hx at lx, tile hx - 1 at lx + TX
  constexpr int LV = LZ * LX;  // one component of a tile region (2D)
  const int qx = wrap_small(j - K.gx0, g.nx);
  const int hx = qx / TX, lx = qx - hx * TX;
  const int txb = hx > 0 ? hx - 1 : K.ntx - 1;
  const bool vb = lx + TX < LX;
  const int xa = hx * 3 * LV + lx;
  const int xb = vb ? txb * 3 * LV + lx + TX : xa;
  const int jw = wrap_small(j, g.nx);
  // tile rows tzw - 2 .. tzw + WT
  constexpr int NTR = WT + 3;
  using A = typename std::conditional<DET, long long, R>::type;  // fold sums
  const A* scratch = reinterpret_cast<const A*>(K.scratch);
  int64_t trow[NTR];
#pragma unroll
  for (int d = 0; d < NTR; d++) {
    int t = tzw + d - 2;
    if (g.periodic_z) t = wrap_small(t, K.ntz);
    else if (t < 0 || t >= K.ntz) t = zero_row;
    if (K.ntiles == 0) t = zero_row;
    trow[d] = (int64_t)t * K.ntx * 3 * LV;
  }
  const int r0 = K.o.rows[0], r1 = K.o.rows[1];
  const int ilo = iw0 - H, ihi = iw0 - H + L - 1;  // rows of the window (unwrapped)
  const bool any_ovf = g.periodic_z ? r1 >= r0 : (ihi >= r0 && ilo <= r1);
#pragma unroll 1
  for (int comp = blockIdx.y * NC; comp < (int)(blockIdx.y + 1) * NC; comp++) {
    const int hz = half_z_j(comp);
    const bool interior = g.periodic_z || (ilo >= 0 && ihi <= row_hi(g, hz));
    // per-lane pointers to row 0 of each candidate tile; rows are then
    // compile-time offsets
    const A* pA[NTR];
    const A* pB[NTR];
#pragma unroll
    for (int d = 0; d < NTR; d++) {
      pA[d] = scratch + trow[d] + comp * LV + xa;
      pB[d] = scratch + trow[d] + comp * LV + xb;
    }
    A va[L];
#pragma unroll
    for (int r = 0; r < L; r++) {
      const int q = r - H;
      const int dt = q >= 0 ? q / TZ : -((TZ - 1 - q) / TZ);
      const int lz = q - dt * TZ;
      A acc = pA[dt + 2][lz * LX];
      const A a1 = pB[dt + 2][lz * LX];
      acc += vb ? a1 : (A)0;
      if (lz + TZ < LZ) {
        const A b0 = pA[dt + 1][(lz + TZ) * LX], b1 = pB[dt + 1][(lz + TZ) * LX];
        acc += b0;
        acc += vb ? b1 : (A)0;
      }
      va[r] = acc;
    }
    if (any_ovf) {
#pragma unroll
      for (int r = 0; r < L; r++) {
        int i = iw0 - H + r;
        if (g.periodic_z) i = wrap_small(i, g.nz);
        if (i >= r0 && i <= r1 && i >= -kGuard && i <= g.nz + kGuard) {
          const int64_t n = (int64_t)(i + kGuard) * g.plane + jw;
          if constexpr (DET) va[r] += K.o.Jq[comp][n];
          else va[r] += K.o.J[comp][n];
        }
      }
    }
    R v[L];
#pragma unroll
    for (int r = 0; r < L; r++) {
      if constexpr (DET) v[r] = (R)((double)va[r] * K.inv_scale);
      else v[r] = va[r];
    }
    if (!interior) {
#pragma unroll
      for (int r = 0; r < L; r++)
        if (!in_domain(g, hz, iw0 - H + r)) v[r] = (R)0;
    }
#pragma unroll
    for (int p = 0; p < NP; p++) {
      const R a = p < fk.passes ? (R)0.25 : (R)fk.a_c;
      const R b = p < fk.passes ? (R)0.5 : (R)fk.b_c;
      R prev = v[0];
#pragma unroll
      for (int r = 1; r < L - 1; r++) {
        const R cur = v[r];
        v[r] = a * prev + b * cur + a * v[r + 1];
        prev = cur;
      }
      if (!interior) {
#pragma unroll
        for (int r = 0; r < L; r++)
          if (!in_domain(g, hz, iw0 - H + r)) v[r] = (R)0;
      }
    }
    R* out = Jf.F[comp];
#pragma unroll
    for (int r = H; r < H + WT * TZ; r++) {
      R x = v[r];
#pragma unroll
      for (int p = 0; p < NP; p++) {
        const R a = p < fk.passes ? (R)0.25 : (R)fk.a_c;
        const R b = p < fk.passes ? (R)0.5 : (R)fk.b_c;
        const R l = __shfl(x, jl), rr = __shfl(x, jr);
        x = a * l + b * x + a * rr;
      }
      const int i = iw0 + r - H;
      if (out_lane && in_domain(g, hz, i)) out[(int64_t)(i + kGuard) * g.plane + j] = x;
    }
  }
}

// 3D fold + filter as three separable sweeps over plain grids, one per axis,
// each applying all of that axis's passes to a register window: z (also folds
// the tile regions and the overflow grid), then x, then y (lane shuffles).
// Lanes run along y, the contiguous axis.  Each sweep reads its input about
// once (window halos) and writes its output once.
template <typename R>
__device__ __forceinline__ R filt_pass_w(const FiltK& fk, int p) {
  return p < fk.passes ? (R)0.25 : (R)fk.a_c;
}
template <typename R>
__device__ __forceinline__ R filt_pass_c(const FiltK& fk, int p) {
  return p < fk.passes ? (R)0.5 : (R)fk.b_c;
}

// z sweep: thread = one (j, k) column and one window of SZ output rows.
template <typename R, int NP, int SZ, int TZ, int TX, int TY, bool DET>
__global__ __launch_bounds__(256) void k_filt3_z(Geo g, FoldK<R> K, FiltK fk, Fields<R> out,
                                                 int nseg) {
  constexpr int H = NP, L = SZ + 2 * H;
  const int comp = blockIdx.z;
  const int hz = half_z_j(comp);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nseg * g.plane) return;
  const int seg = (int)(t / g.plane);
  const int q = (int)(t - (int64_t)seg * g.plane);
  const int j = q / g.ny, k = q - j * g.ny;
  const int i0 = seg * SZ;
  R v[L];
#pragma unroll
  for (int r = 0; r < L; r++) {
    const int i = i0 - H + r;
    v[r] = (g.periodic_z || in_domain(g, hz, i)) ? fold_at<R, 3, TZ, TX, TY, DET>(K, g, comp, i, j, k)
                                                 : (R)0;
  }
#pragma unroll
  for (int p = 0; p < NP; p++) {
    const R a = filt_pass_w<R>(fk, p), b = filt_pass_c<R>(fk, p);
    R prev = v[0];
#pragma unroll
    for (int r = 1; r < L - 1; r++) {
      const R cur = v[r];
      v[r] = a * prev + b * cur + a * v[r + 1];
      prev = cur;
    }
    if (!g.periodic_z) {
#pragma unroll
      for (int r = 0; r < L; r++)
        if (!in_domain(g, hz, i0 - H + r)) v[r] = (R)0;
    }
  }
  R* o = out.F[comp];
#pragma unroll
  for (int r = H; r < H + SZ; r++) {
    const int i = i0 + r - H;
    if (in_domain(g, hz, i)) o[(int64_t)(i + kGuard) * g.plane + q] = v[r];
  }
}

// z sweep with the fold, open z, windows aligned to the tile rows: window
// rows start where a tile row's region starts (row gz0 + m TZ), so that each
// window row's local row in a region, and with it the set of tile rows whose
// regions hold it, are compile-time constants.  Along x the candidates are
// the same for a whole thread column (NBX: 3 where some lane of the wave
// needs a third, else 2).  A candidate is read only where the node lies in
// its region's box of nonzero nodes.  Same sums, in the same order, as
// fold_at.
template <typename R, int NP, int SZ, int TZ, int TX, int TY, int LZ, int LX, int LY, bool DET,
          int NBX>
__device__ __forceinline__ void filt3_z_aligned_body(const Geo& g, const FoldK<R>& K,
                                                     const FiltK& fk, Fields<R>& out, int comp,
                                                     int i0, int m, int q, int j, int k) {
  constexpr int H = NP, L = SZ + 2 * H;
  constexpr int LV = LZ * LX * LY;
  using A = typename std::conditional<DET, long long, R>::type;
  const A* scratch = reinterpret_cast<const A*>(K.scratch);
  const int hz = half_z_j(comp);
  // x and y candidates of this column: tile within a tile row, and whether
  // the column lies in that tile's region
  const int qx = wrap_small(j - K.gx0, g.nx), qy = wrap_small(k - K.gy0, g.ny);
  const int hx = qx / TX, lx = qx - hx * TX;
  const int hy = qy / TY, ly = qy - hy * TY;
  int tin[NBX][3];
  bool val[NBX][3];
#pragma unroll
  for (int b = 0; b < NBX; b++) {
    int tx = hx - b;
    if (tx < 0) tx += K.ntx;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      int ty = hy - c;
      if (ty < 0) ty += K.nty;
      val[b][c] = lx + b * TX < LX && ly + c * TY < LY;
      tin[b][c] = tx * K.nty + ty;
    }
  }
  // Tile rows m - 2 .. m + (L - 1) / TZ; row d holds window row r at local
  // z r - (d - 2) TZ.  Taken from the top row down, so that each window row
  // adds its candidates in the order of fold_at (z, then x, then y); only
  // nodes inside a region's box are read.
  constexpr int NTR = (L - 1) / TZ + 3;
  const int row_tiles = K.ntx * K.nty;
  A acc[L];
#pragma unroll
  for (int r = 0; r < L; r++) acc[r] = (A)0;
#pragma unroll
  for (int d = NTR - 1; d >= 0; d--) {
    const int tr = m + d - 2;
    const bool row_ok = tr >= 0 && tr < K.ntz;
#pragma unroll
    for (int b = 0; b < NBX; b++)
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const bool ok = row_ok && val[b][c];
        const int t = ok ? tr * row_tiles + tin[b][c] : 0;
        const unsigned w = K.box[t];
        const RegionBox bx = unpack_box(ok ? w : 0u);
        const int ox = lx + b * TX - bx.x0, oy = ly + c * TY - bx.y0;
        const bool in_xy = (unsigned)ox < (unsigned)bx.nx && (unsigned)oy < (unsigned)bx.ny;
        const int64_t base = (int64_t)t * 3 * LV + comp * bx.vol() + ox * bx.ny + oy;
        const int zs = bx.nx * bx.ny;
#pragma unroll
        for (int r = 0; r < L; r++) {
          const int lz = r - (d - 2) * TZ;
          if (lz < 0 || lz >= LZ) continue;  // compile-time
          const int oz = lz - bx.z0;
          if (in_xy && (unsigned)oz < (unsigned)bx.nz) acc[r] += scratch[base + oz * zs];
        }
      }
  }
  const int r0 = K.o.rows[0], r1 = K.o.rows[1];
  R v[L];
#pragma unroll
  for (int r = 0; r < L; r++) {
    A a = acc[r];
    const int i = i0 - H + r;
    if (i >= r0 && i <= r1 && i >= -kGuard && i <= g.nz + kGuard) {
      const int64_t n = (int64_t)(i + kGuard) * g.plane + q;
      if constexpr (DET) a += K.o.Jq[comp][n];
      else a += K.o.J[comp][n];
    }
    R x;
    if constexpr (DET) x = (R)((double)a * K.inv_scale);
    else x = a;
    v[r] = in_domain(g, hz, i) ? x : (R)0;
  }
#pragma unroll
  for (int p = 0; p < NP; p++) {
    const R a = filt_pass_w<R>(fk, p), b = filt_pass_c<R>(fk, p);
    R prev = v[0];
#pragma unroll
    for (int r = 1; r < L - 1; r++) {
      const R cur = v[r];
      v[r] = a * prev + b * cur + a * v[r + 1];
      prev = cur;
    }
#pragma unroll
    for (int r = 0; r < L; r++)
      if (!in_domain(g, hz, i0 - H + r)) v[r] = (R)0;
  }
  R* o = out.F[comp];
#pragma unroll
  for (int r = H; r < H + SZ; r++) {
    const int i = i0 + r - H;
    if (in_domain(g, hz, i)) o[(int64_t)(i + kGuard) * g.plane + q] = v[r];
  }
}

template <typename R, int NP, int SZ, int TZ, int TX, int TY, int LZ, int LX, int LY, bool DET>
__global__ __launch_bounds__(256) void k_filt3_z_aligned(Geo g, FoldK<R> K, FiltK fk,
                                                         Fields<R> out, int nseg, int i0_first,
                                                         int m_first) {
  static_assert(SZ % TZ == 0, "windows of whole tile rows");
  const int comp = blockIdx.z;
  // blocks dealt XCD-aware (a slab of windows per XCD), so that the
  // neighbouring box rows that share cache lines share an L2: 0.92 against
  // 1.96 GB fetched per launch at 512 x 128 x 128, 27 us less per step
  const int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const bool live = t < (int64_t)nseg * g.plane;
  const int tt = live ? (int)t : 0;
  const int seg = tt / g.plane;
  const int q = tt - seg * g.plane;
  const int j = q / g.ny, k = q - j * g.ny;
  const int i0 = i0_first + seg * SZ, m = m_first + seg * (SZ / TZ);
  const int qx = wrap_small(j - K.gx0, g.nx);
  const bool third = live && qx % TX + 2 * TX < LX;
  if (!live) return;
  if (__any(third))
    filt3_z_aligned_body<R, NP, SZ, TZ, TX, TY, LZ, LX, LY, DET, 3>(g, K, fk, out, comp, i0, m,
                                                                    q, j, k);
  else
    filt3_z_aligned_body<R, NP, SZ, TZ, TX, TY, LZ, LX, LY, DET, 2>(g, K, fk, out, comp, i0, m,
                                                                    q, j, k);
}

// x sweep (periodic): thread = one (i, k) line and one window of SX outputs.
template <typename R, int NP, int SX>
__global__ __launch_bounds__(256) void k_filt3_x(Geo g, FiltK fk, Fields<R> in, Fields<R> out,
                                                 int nseg) {
  constexpr int H = NP, L = SX + 2 * H;
  const int comp = blockIdx.z;
  const int hz = half_z_j(comp);
  const int nrow = row_hi(g, hz) + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nrow * nseg * g.ny) return;
  const int k = (int)(t % g.ny);
  const int64_t rest = t / g.ny;
  const int seg = (int)(rest % nseg), i = (int)(rest / nseg);
  const int j0 = seg * SX;
  const R* a_in = in.F[comp] + (int64_t)(i + kGuard) * g.plane + k;
  R v[L];
#pragma unroll
  for (int r = 0; r < L; r++) v[r] = a_in[(int64_t)wrap_small(j0 - H + r, g.nx) * g.ny];
#pragma unroll
  for (int p = 0; p < NP; p++) {
    const R a = filt_pass_w<R>(fk, p), b = filt_pass_c<R>(fk, p);
    R prev = v[0];
#pragma unroll
    for (int r = 1; r < L - 1; r++) {
      const R cur = v[r];
      v[r] = a * prev + b * cur + a * v[r + 1];
      prev = cur;
    }
  }
  R* o = out.F[comp] + (int64_t)(i + kGuard) * g.plane + k;
#pragma unroll
  for (int r = H; r < H + SX; r++) {
    const int j = j0 + r - H;
    if (j < g.nx) o[(int64_t)j * g.ny] = v[r];
  }
}

// y sweep (periodic): one wave per (i, j) line and window of 64 - 2 NP outputs.
template <typename R, int NP>
__global__ __launch_bounds__(256) void k_filt3_y(Geo g, FiltK fk, Fields<R> in, Fields<R> out,
                                                 int nseg) {
  constexpr int H = NP, FY = 64 - 2 * H;
  const int comp = blockIdx.z;
  const int hz = half_z_j(comp);
  const int nrow = row_hi(g, hz) + 1;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) +
                                                     (threadIdx.x >> 6)));
  if (w >= nrow * g.nx * nseg) return;  // the whole wave leaves together
  const int seg = w % nseg, line = w / nseg;
  const int i = line / g.nx, j = line - i * g.nx;
  const int k = seg * FY - H + lane;
  const int64_t base = ((int64_t)(i + kGuard) * g.nx + j) * g.ny;
  R x = in.F[comp][base + wrap_small(k, g.ny)];
  const int kl = lane == 0 ? 63 : lane - 1, kr = lane == 63 ? 0 : lane + 1;
#pragma unroll
  for (int p = 0; p < NP; p++) {
    const R a = filt_pass_w<R>(fk, p), b = filt_pass_c<R>(fk, p);
    const R l = __shfl(x, kl), r = __shfl(x, kr);
    x = a * l + b * x + a * r;
  }
  if (lane >= H && lane < 64 - H && k < g.ny) out.F[comp][base + k] = x;
}

// y sweep (periodic) over whole lines, for ny = 64 M: one wave per (i, j)
// line, lane l holding nodes l + 64 m; the neighbours across lanes 0 and 63
// come from the adjacent register (wrapping at the line's ends).  The same
// arithmetic per node as k_filt3_y, with a third of its waves and no halo
// reloads.
template <typename R, int NP, int M>
__global__ __launch_bounds__(256) void k_filt3_y_line(Geo g, FiltK fk, Fields<R> in,
                                                      Fields<R> out) {
  const int comp = blockIdx.z;
  const int hz = half_z_j(comp);
  const int nrow = row_hi(g, hz) + 1;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) +
                                                     (threadIdx.x >> 6)));
  if (w >= nrow * g.nx) return;  // the whole wave leaves together
  const int i = w / g.nx, j = w - i * g.nx;
  const int64_t base = ((int64_t)(i + kGuard) * g.nx + j) * g.ny;
  R x[M];
#pragma unroll
  for (int m = 0; m < M; m++) x[m] = in.F[comp][base + m * 64 + lane];
  const int kl = lane == 0 ? 63 : lane - 1, kr = lane == 63 ? 0 : lane + 1;
#pragma unroll
  for (int p = 0; p < NP; p++) {
    const R a = filt_pass_w<R>(fk, p), b = filt_pass_c<R>(fk, p);
    R l[M], r[M];
#pragma unroll
    for (int m = 0; m < M; m++) {
      l[m] = __shfl(x[m], kl);
      r[m] = __shfl(x[m], kr);
    }
#pragma unroll
    for (int m = 0; m < M; m++) {
      // lane 0: node 64 m - 1 is lane 63 of register m - 1; lane 63: node
      // 64 m + 64 is lane 0 of register m + 1
      const R left = lane == 0 ? l[(m + M - 1) % M] : l[m];
      const R right = lane == 63 ? r[(m + 1) % M] : r[m];
      x[m] = a * left + b * x[m] + a * right;
    }
  }
#pragma unroll
  for (int m = 0; m < M; m++) out.F[comp][base + m * 64 + lane] = x[m];
}

// Clear the overflow rows that the global path touched this step.
template <typename R, bool DET>
__global__ __launch_bounds__(256) void k_ovf_clear(Geo g, Ovf<R> o) {
  int r0 = o.rows[0], r1 = o.rows[1];
  if (r1 < r0) return;
  if (r0 < -kGuard) r0 = -kGuard;
  if (r1 > g.nz + kGuard) r1 = g.nz + kGuard;
  int64_t n = (int64_t)(r1 - r0 + 1) * g.plane;
  int64_t base = (int64_t)(r0 + kGuard) * g.plane;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    for (int c = 0; c < 3; c++) {
      if constexpr (DET) o.Jq[c][base + v] = 0;
      else o.J[c][base + v] = (R)0;
    }
  }
}

__global__ void k_ovf_reset(int* rows, int* nstrag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    rows[0] = 0x7fffffff;
    rows[1] = -0x7fffffff;
    *nstrag = 0;
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

// Node (i, j, k) of a Yee update: row i = blockIdx.y, plane index from x;
// the storage index of a neighbour one node away along each axis (periodic
// in x, y, and in z when the grid is; open z reads the guard rows).
struct YeeNode {
  int i, j, k;
  int64_t n;            // this node
  int64_t zp, zm;       // rows i + 1, i - 1
  int64_t xp, xm, yp, ym;
};
__device__ __forceinline__ bool yee_node(const Geo& g, YeeNode& d) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.plane) return false;
  d.i = blockIdx.y;
  d.j = q / g.ny;
  d.k = q - d.j * g.ny;
  const int64_t row = (int64_t)(d.i + kGuard) * g.plane;
  d.n = row + q;
  int ip = d.i + 1, im = d.i - 1;
  if (g.periodic_z) {
    if (ip == g.nz) ip = 0;
    if (im < 0) im = g.nz - 1;
  }
  d.zp = (int64_t)(ip + kGuard) * g.plane + q;
  d.zm = (int64_t)(im + kGuard) * g.plane + q;
  const int jp = d.j + 1 == g.nx ? 0 : d.j + 1, jm = d.j == 0 ? g.nx - 1 : d.j - 1;
  const int kp = d.k + 1 == g.ny ? 0 : d.k + 1, km = d.k == 0 ? g.ny - 1 : d.k - 1;
  d.xp = row + (int64_t)jp * g.ny + d.k;
  d.xm = row + (int64_t)jm * g.ny + d.k;
  d.yp = row + (int64_t)d.j * g.ny + kp;
  d.ym = row + (int64_t)d.j * g.ny + km;
  return true;
}

// Launched with grid (cdiv(plane, 256), rows): rows nz + 1 (open z) or nz.
template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_yee_b(Geo g, YeeK<R> Y) {
  YeeNode d;
  if (!yee_node(g, d)) return;
  const int64_t n = d.n;
  const R* Ex = Y.E[0];
  const R* Ey = Y.E[1];
  const R* Ez = Y.E[2];
  R ey = Ey[n];
  if (d.i <= row_hi(g, 1)) {
    R dEz_dy = DIM == 3 ? (Ez[d.yp] - Ez[n]) * Y.idy : (R)0;
    Y.B[0][n] += Y.h * ((Ey[d.zp] - ey) * Y.idz - dEz_dy);
    Y.B[1][n] += Y.h * ((Ez[d.xp] - Ez[n]) * Y.idx - (Ex[d.zp] - Ex[n]) * Y.idz);
  }
  R dEx_dy = DIM == 3 ? (Ex[d.yp] - Ex[n]) * Y.idy : (R)0;
  Y.B[2][n] += Y.h * (dEx_dy - (Ey[d.xp] - ey) * Y.idx);
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_yee_e(Geo g, YeeK<R> Y) {
  YeeNode d;
  if (!yee_node(g, d)) return;
  const int64_t n = d.n;
  const int i = d.i;
  const R* Bx = Y.B[0];
  const R* By = Y.B[1];
  const R* Bz = Y.B[2];
  bool open = !g.periodic_z;
  if (i <= row_hi(g, 1)) {
    R dBx_dy = DIM == 3 ? (Bx[n] - Bx[d.ym]) * Y.idy : (R)0;
    Y.E[2][n] += Y.h * ((By[n] - By[d.xm]) * Y.idx - dBx_dy - Y.J[2][n]);
  }
  if (open && (i == 0 || i == g.nz)) return;  // Mur planes
  if (open && (i == 1 || i == g.nz - 1)) {
    int r = i == 1 ? 0 : 1;
    int64_t q = n - (int64_t)(i + kGuard) * g.plane;
    Y.save[(r * 2 + 0) * g.plane + q] = Y.E[0][n];
    Y.save[(r * 2 + 1) * g.plane + q] = Y.E[1][n];
  }
  R dBz_dy = DIM == 3 ? (Bz[n] - Bz[d.ym]) * Y.idy : (R)0;
  Y.E[0][n] += Y.h * (dBz_dy - (By[n] - By[d.zm]) * Y.idz - Y.J[0][n]);
  Y.E[1][n] += Y.h * ((Bx[n] - Bx[d.zm]) * Y.idz - (Bz[n] - Bz[d.xm]) * Y.idx - Y.J[1][n]);
}

// 2D Yee step fused into one kernel: B half step, E step with the filtered
// current, Mur at open z ends, B half step -- the same updates as k_yee_b,
// k_yee_e, k_mur, k_yee_b, node by node.  Each lane owns one x column and a
// wave marches along z through a band of rows, keeping the few rows each
// update needs in registers; x neighbours come from the adjacent lanes.  The
// dependency cone of one output node spans one column to the left and two
// to the right, so a wave holds 64 consecutive columns and writes the 61
// inner ones.  The kernel reads E, B from one set of arrays and writes the
// other (neighbouring bands read its halo rows), so the caller swaps the two
// sets afterwards.
template <typename R>
struct YeeF {
  const R* E[3];
  const R* B[3];
  const R* J[3];
  R* Eo[3];
  R* Bo[3];
  R idz, idx;
  R h1, h;   // dt / 2 and dt
  R mur;
};

constexpr int kYeeCols = 61;  // output columns per wave

template <typename R>
__device__ __forceinline__ R lane_next(R v) { return __shfl_down(v, 1, 64); }
template <typename R>
__device__ __forceinline__ R lane_prev(R v) { return __shfl_up(v, 1, 64); }

// Waves are numbered band-major (band = wave / nwx); band b covers rows
// [b tz, (b + 1) tz), the last band also the remainder.
template <typename R>
__global__ __launch_bounds__(256) void k_yee2d(Geo g, YeeF<R> Y, int nwx, int tz,
                                                int nband) {
  const int lane = threadIdx.x & 63;
  // XCD-aware: neighbouring bands (which read each other's halo rows) share an L2
  const int wid = xcd_remap(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int band = wid / nwx, w = wid - band * nwx;
  if (band >= nband) return;  // whole wave
  const bool open = !g.periodic_z;
  const int nrow = open ? g.nz + 1 : g.nz;
  const int rh1 = row_hi(g, 1);
  const int i0 = band * tz, i1 = band == nband - 1 ? nrow : i0 + tz;
  const int cu = w * kYeeCols + lane - 1;  // unwrapped column of this lane
  const int j = wrapi(cu, g.nx);
  const bool out = lane >= 1 && lane <= kYeeCols && cu < g.nx;
  // every row touched lies in [i0 - 2, i1 + 2] within storage (open z) or
  // wraps (periodic z)
  auto at = [&](int i) -> int64_t {
    const int r = open ? i : wrapi(i, g.nz);
    return (int64_t)(r + kGuard) * g.nx + j;
  };
  const R idz = Y.idz, idx = Y.idx, h1 = Y.h1, h = Y.h, m = Y.mur;
  auto in_b = [&](int i) { return !open || (i >= 0 && i <= rh1); };    // Bx, By, Ez
  auto in_z = [&](int i) { return !open || (i >= 0 && i < nrow); };    // Bz
  auto in_e = [&](int i) { return !open || (i >= 1 && i <= g.nz - 1); };  // Ex, Ey
  struct V3 { R x, y, z; };
  auto ld = [&](const R* const* A, int64_t n) { return V3{A[0][n], A[1][n], A[2][n]}; };
  // B half step of row i from E rows i (with its right neighbours) and i + 1
  auto bhalf = [&](V3 b, int i, V3 e, V3 e1) {
    const R ezr = lane_next(e.z), eyr = lane_next(e.y);
    if (in_b(i)) {
      b.x += h1 * ((e1.y - e.y) * idz);
      b.y += h1 * ((ezr - e.z) * idx - (e1.x - e.x) * idz);
    }
    if (in_z(i)) b.z += h1 * (-(eyr - e.y) * idx);
    return b;
  };
  // E step of row i from B rows i (with its left neighbours) and i - 1
  auto estep = [&](V3 e, int i, V3 b, V3 bm, V3 jc) {
    const R byl = lane_prev(b.y), bzl = lane_prev(b.z);
    if (in_b(i)) e.z += h * ((b.y - byl) * idx - jc.z);
    if (in_e(i)) {
      e.x += h * (-(b.y - bm.y) * idz - jc.x);
      e.y += h * ((b.x - bm.x) * idz - (b.z - bzl) * idx - jc.y);
    }
    return e;
  };
  // prologue: B half on rows i0 - 2 and i0 - 1, E step on row i0 - 1
  V3 eo_m = ld(Y.E, at(i0 - 2)), eo = ld(Y.E, at(i0 - 1)), eo_p = ld(Y.E, at(i0));
  V3 bh_m = bhalf(ld(Y.B, at(i0 - 2)), i0 - 2, eo_m, eo);
  V3 bh = bhalf(ld(Y.B, at(i0 - 1)), i0 - 1, eo, eo_p);
  V3 en = estep(eo, i0 - 1, bh, bh_m, ld(Y.J, at(i0 - 1)));
  // Mur rewrites row 0 at i = 1 and row nz at i = nz, inside the loop, from
  // the previous row's old and new E (the prologue's for the first i)
  V3 nb = ld(Y.B, at(i0)), nj = ld(Y.J, at(i0)), ne = ld(Y.E, at(i0 + 1));
  for (int i = i0; i <= i1; i++) {
    // row i: old E (eo_p), B, J; old E of row i + 1 (ne)
    const V3 eo_c = eo_p, bi = nb, ji = nj, e1 = ne;
    if (i < i1) {
      nb = ld(Y.B, at(i + 1));
      nj = ld(Y.J, at(i + 1));
      ne = ld(Y.E, at(i + 2));
    }
    const V3 bh_c = bhalf(bi, i, eo_c, e1);
    V3 en_c = estep(eo_c, i, bh_c, bh, ji);
    if (open && i == 1) {  // Mur at z = 0 rewrites row 0 from row 1
      en.x = eo_c.x + m * (en_c.x - eo.x);
      en.y = eo_c.y + m * (en_c.y - eo.y);
    }
    if (open && i == g.nz) {  // Mur at z = nz rewrites row nz from row nz - 1
      en_c.x = eo.x + m * (en.x - eo_c.x);
      en_c.y = eo.y + m * (en.y - eo_c.y);
    }
    // B half step of row i - 1 with the new E, then store row i - 1
    const V3 bf = bhalf(bh, i - 1, en, en_c);
    if (i > i0 && out) {
      const int64_t n = at(i - 1);
      Y.Eo[0][n] = en.x;
      Y.Eo[1][n] = en.y;
      Y.Eo[2][n] = en.z;
      Y.Bo[0][n] = bf.x;
      Y.Bo[1][n] = bf.y;
      Y.Bo[2][n] = bf.z;
    }
    eo = eo_c;
    eo_p = e1;
    bh = bh_c;
    en = en_c;
  }
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

// --------------------------------------------------------------------------
// Laser antenna: the current sheet J_y = -2 E_y'(t', z_a, x[, y]) / dz on one
// grid row, which radiates the boosted laser's E_y into both directions (in
// 1D vacuum a surface current K radiates E_y = -K/2 on either side; a sheet on
// one row carries K = J_y dz).  Added to the filtered current; t' is the
// step's mid time, the laser is evaluated at the boosted event (t', z_a) as in
// k_laser_a, with its transverse images.  One thread per node of the row.
// --------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_antenna(Geo g, LaserK K, double tp, double zp, int row,
                                                 R* Jy) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.plane) return;
  const int j = (int)(q / g.ny), k = (int)(q - (int64_t)j * g.ny);
  const double x = (double)j * K.dx - K.xa;
  const double y = K.dim == 3 ? ((double)k + 0.5) * K.dy - K.ya : 0.0;
  const double xi = K.gomb * (zp - tp) - K.zc;
  const double zeta = K.gamma_b * zp + K.gbeta * tp - K.zf;
  const int my = K.dim == 3 ? K.iy : 0;
  double Es = 0.0;
  for (int mx = -K.ix; mx <= K.ix; mx++)
    for (int mm = -my; mm <= my; mm++) {
      double a, dxi, dze;
      lab_potential(K, xi, zeta, x + mx * K.Lx, y + mm * K.Ly, a, dxi, dze);
      Es += K.gomb * dxi - K.gbeta * dze;
    }
  Jy[gidx(g, row, j, k)] += (R)(-2.0 * Es / K.dz);
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
