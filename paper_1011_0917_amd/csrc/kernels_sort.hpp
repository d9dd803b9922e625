// kernels_sort.hpp -- particle sort by co-moving tile-major cell key, ties by
// id: count (atomic rank per key), exclusive scan, scatter, per-cell sort
// by id (makes the order unique), interleave of each tile by
// rank within cell, permute, tile starts.
#pragma once

#include "device_common.hpp"
#include "kernels_particles.hpp"

namespace bfpic {

struct SortK {
  int TZ, TX, TY;
  int ntz, ntx, nty;
  int zc0;    // co-moving z cell of tile row 0
  int nkeys;  // ntz*ntx*nty*TZ*TX*TY; removed particles get key nkeys
};

// Key of the electron's co-moving cell (its partner's birth cell plus the
// floor of birth offset + displacement), clamped into the tile rows along z.
template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_sort_keys(PSoA<R> S, LatticeP L, Geo g, SortK K,
                                                   const int* counts, int* key, int* rank,
                                                   int* cnt) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= counts[0]) return;
  int id = S.id[p];
  int kk = K.nkeys;
  if (id >= 0) {
    Birth b = decode_id(L, id);
    R oz = birth_offset<R>(L, id, 0) + S.xi[0][p];
    R ox = birth_offset<R>(L, id, 1) + S.xi[1][p];
    int kz = b.k + (int)floor(oz);
    int kx = wrapi(b.j + (int)floor(ox), g.nx);
    int ky = 0;
    if (DIM == 3) {
      R oy = birth_offset<R>(L, id, 2) + S.xi[2][p];
      ky = wrapi(b.l + (int)floor(oy), g.ny);
    }
    if (g.periodic_z) kz = wrapi(kz, g.nz);
    int rz = kz - K.zc0;
    if (rz < 0) rz = 0;
    if (rz >= K.ntz * K.TZ) rz = K.ntz * K.TZ - 1;
    int tile = ((rz / K.TZ) * K.ntx + kx / K.TX) * K.nty + ky / K.TY;
    int loc = ((rz % K.TZ) * K.TX + kx % K.TX) * K.TY + ky % K.TY;
    kk = tile * (K.TZ * K.TX * K.TY) + loc;
  }
  key[p] = kk;
  rank[p] = atomicAdd(&cnt[kk], 1);
}

// Exclusive scan of n ints in three launches (block scans of 4096, scan of
// the block sums in one workgroup, add-back).
constexpr int kScanBlock = 1024, kScanPer = 4;

__global__ __launch_bounds__(kScanBlock) void k_scan_blocks(const int* in, int* out, int* bsum,
                                                            int64_t n) {
  __shared__ int s[kScanBlock];
  int64_t base = ((int64_t)blockIdx.x * kScanBlock + threadIdx.x) * kScanPer;
  int v[kScanPer];
  int tot = 0;
  for (int m = 0; m < kScanPer; m++) {
    int64_t q = base + m;
    v[m] = q < n ? in[q] : 0;
    tot += v[m];
  }
  s[threadIdx.x] = tot;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int run = s[threadIdx.x] - tot;
  for (int m = 0; m < kScanPer; m++) {
    int64_t q = base + m;
    if (q < n) out[q] = run;
    run += v[m];
  }
  if (threadIdx.x == kScanBlock - 1) bsum[blockIdx.x] = s[threadIdx.x];
}

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(int* bsum, int nb) {
  __shared__ int s[kScanBlock];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += kScanBlock) {
    int q = base + threadIdx.x;
    int v = q < nb ? bsum[q] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
      int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (q < nb) bsum[q] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == kScanBlock - 1) carry += s[threadIdx.x];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_scan_add(int* out, const int* bsum, int64_t n) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  out[q] += bsum[q / (kScanBlock * kScanPer)];
}

__global__ __launch_bounds__(256) void k_sort_scatter(const int* counts, const int* key,
                                                      const int* rank, const int* off,
                                                      int* perm) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= counts[0]) return;
  perm[off[key[p]] + rank[p]] = p;
}

// Within each key the atomic ranks are arbitrary: order them by id.  A cell
// of up to kCellReg particles is sorted in registers (its slots and ids are
// loaded in two independent rounds, then an odd-even transposition network
// orders them); a fuller one by insertion through memory.  Ids are distinct,
// so both give the same order.
constexpr int kCellReg = 32;

__global__ __launch_bounds__(256) void k_sort_cells(const int* off, const int* id, int* perm,
                                                    int nkeys) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nkeys) return;
  int a = off[c], b = off[c + 1];
  const int n = b - a;
  if (n <= 1) return;
  if (n <= kCellReg) {
    int pv[kCellReg], iv[kCellReg];
#pragma unroll
    for (int m = 0; m < kCellReg; m++) pv[m] = m < n ? perm[a + m] : 0;
#pragma unroll
    for (int m = 0; m < kCellReg; m++) iv[m] = m < n ? id[pv[m]] : INT_MAX;
    // n passes of odd-even transposition sort n entries; the padding
    // (INT_MAX) stays at the end
    for (int pass = 0; pass < n; pass++) {
#pragma unroll
      for (int m = 0; m + 1 < kCellReg; m += 2) {
        const int q = m + (pass & 1);
        if (q + 1 < kCellReg && iv[q] > iv[q + 1]) {
          const int ti = iv[q], tp = pv[q];
          iv[q] = iv[q + 1];
          pv[q] = pv[q + 1];
          iv[q + 1] = ti;
          pv[q + 1] = tp;
        }
      }
    }
#pragma unroll
    for (int m = 0; m < kCellReg; m++)
      if (m < n) perm[a + m] = pv[m];
    return;
  }
  for (int x = a + 1; x < b; x++) {
    int pv = perm[x];
    int iv = id[pv];
    int y = x - 1;
    while (y >= a && id[perm[y]] > iv) {
      perm[y + 1] = perm[y];
      y--;
    }
    perm[y + 1] = pv;
  }
}

// Within each tile, reorder the (cell, id)-sorted particles by (rank within
// their cell, cell): position of rank r of cell c is
//   sum_{r' < r} #{cells with more than r' particles} + #{c' < c with more than r}.
// Consecutive particles then sit in distinct cells, so the lanes of a wave
// add their currents to distinct LDS addresses.  One workgroup per tile of
// cpt <= kInterleaveCells cells.
constexpr int kInterleaveCells = 512;

__global__ __launch_bounds__(256) void k_sort_interleave(const int* off, const int* perm,
                                                         int* out, int cpt) {
  __shared__ int n[kInterleaveCells];
  __shared__ int sc[256];
  __shared__ int red;
  const int t = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * cpt;
  const int base = off[k0];
  if (t == 0) red = 0;
  __syncthreads();
  int mx = 0;
  for (int c = t; c < cpt; c += 256) {
    n[c] = off[k0 + c + 1] - off[k0 + c];
    mx = max(mx, n[c]);
  }
  atomicMax(&red, mx);
  __syncthreads();
  const int maxn = red;
  // each thread owns cells [t * per, t * per + per)
  const int per = (cpt + 255) / 256;
  int S = 0;
  for (int r = 0; r < maxn; r++) {
    int cntv = 0;
    for (int m = 0; m < per; m++) {
      const int c = t * per + m;
      cntv += (c < cpt && n[c] > r) ? 1 : 0;
    }
    sc[t] = cntv;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const int v = t >= o ? sc[t - o] : 0;
      __syncthreads();
      sc[t] += v;
      __syncthreads();
    }
    int pos = S + sc[t] - cntv;  // exclusive prefix
    const int Nr = sc[255];
    for (int m = 0; m < per; m++) {
      const int c = t * per + m;
      if (c < cpt && n[c] > r) {
        out[base + pos] = perm[off[k0 + c] + r];
        pos++;
      }
    }
    S += Nr;
    __syncthreads();
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_permute(PSoA<R> src, PSoA<R> dst, const int* perm,
                                                 const int* off_end) {
  int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= *off_end) return;
  int s = perm[d];
  dst.id[d] = src.id[s];
  dst.xi[0][d] = src.xi[0][s];
  dst.xi[1][d] = src.xi[1][s];
  if (src.xi[2]) dst.xi[2][d] = src.xi[2][s];
  dst.du[0][d] = src.du[0][s];
  dst.du[1][d] = src.du[1][s];
  dst.du[2][d] = src.du[2][s];
  dst.w[d] = src.w[s];
}

__global__ __launch_bounds__(256) void k_tile_starts(const int* off, int* start, int ntiles,
                                                     int cpt, int* counts, int nkeys) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t <= ntiles) start[t] = off[(int64_t)t * cpt];
  if (t == 0) {
    counts[0] = off[nkeys];
    counts[1] = off[nkeys];
  }
}

// Largest-first dispatch order of the tiles (longest-processing-time list
// scheduling): once the wake bunches the plasma, a few tiles hold several
// times the mean count and would otherwise finish last.  Tiles are binned by
// particle count (bin width 2^shift) and listed from the fullest bin down.
// One workgroup.  The order inside a bin is arbitrary: every tile owns its
// scratch region, so the order changes no result.
constexpr int kOrderBins = 256;

__global__ __launch_bounds__(1024) void k_tile_order(const int* start, int ntiles, int shift,
                                                     int* order) {
  __shared__ int cnt[kOrderBins];
  for (int b = threadIdx.x; b < kOrderBins; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  auto bin = [&](int t) {
    const int b = (start[t + 1] - start[t]) >> shift;
    return kOrderBins - 1 - (b < kOrderBins - 1 ? b : kOrderBins - 1);
  };
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) atomicAdd(&cnt[bin(t)], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int b = 0; b < kOrderBins; b++) {
      const int c = cnt[b];
      cnt[b] = s;
      s += c;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) order[atomicAdd(&cnt[bin(t)], 1)] = t;
}

}  // namespace bfpic
