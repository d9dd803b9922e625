// bfpic.hip -- host side of the C ABI declared in include/bfpic.h.
//
// The context borrows one caller-owned device workspace, carves it into the
// field, particle, sort, tile and diagnostic buffers, and enqueues every step
// on the caller's stream with no host synchronisation inside pic_step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bfpic.h"
#include "device_common.hpp"
#include "kernels_diag.hpp"
#include "kernels_fields.hpp"
#include "kernels_particles.hpp"
#include "kernels_sort.hpp"
#include "kernels_adjoint.hpp"
#include "kernels_lab.hpp"
#include "kernels_witness.hpp"

using namespace bfpic;

// ---------------------------------------------------------------------------
// Static device scratch of diagnostics_noalloc: the block partials of its
// reductions, its final values and its non-finite flag.  Each device that
// runs the library holds one copy until the process ends; every call on a
// device shares it (calls that overlap on one device race).  Host code never
// passes the array's name to a kernel: it uses the address that
// hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
constexpr int64_t kStaticScratchBytes = 32768;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on device dev (which must be current), resolved once.
static hipError_t static_scratch_of(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Boost helper (host FP64).  Frame change along +z by rapidity artanh(beta_b).
// ---------------------------------------------------------------------------
extern "C" double bfpic_beta(double gamma) { return std::sqrt(gamma * gamma - 1.0) / gamma; }
extern "C" double bfpic_drift_u(double gamma_b) { return -std::sqrt(gamma_b * gamma_b - 1.0); }
extern "C" double bfpic_group_gamma(double n_lab) { return 1.0 / std::sqrt(n_lab); }
extern "C" double bfpic_boosted_group_beta(double gamma_b, double n_lab) {
  // (beta_g - beta_b) / (1 - beta_g beta_b) with
  // beta_g - beta_b = (gamma_b^-2 - gamma_g^-2) / (beta_g + beta_b) and
  // 1 - beta_g beta_b = (gamma_g^-2 + gamma_b^-2 + (beta_g - beta_b)^2) / 2
  double gg = bfpic_group_gamma(n_lab);
  double bg = bfpic_beta(gg), bb = bfpic_beta(gamma_b);
  double a = 1.0 / (gamma_b * gamma_b), c = 1.0 / (gg * gg);
  double diff = (a - c) / (bg + bb);
  return diff / (0.5 * (c + a + diff * diff));
}
extern "C" double bfpic_boosted_dz(double gamma_b, double lambda0, double cells) {
  return gamma_b * (1.0 + bfpic_beta(gamma_b)) * lambda0 / cells;
}
extern "C" double bfpic_yee_dt(int32_t dim, double dz, double dx, double dy, double cfl) {
  double s = 1.0 / (dz * dz) + 1.0 / (dx * dx) + (dim == 3 ? 1.0 / (dy * dy) : 0.0);
  return cfl / std::sqrt(s);
}

// ---------------------------------------------------------------------------
// Tile shapes: 2D 16 x 32 cells, 3D 8 x 8 x 8 cells; excursion margin 1 cell.
// ---------------------------------------------------------------------------
constexpr int kExc = 1;
constexpr int kT2Z = 16, kT2X = 32;
constexpr int kT3 = 8;
constexpr int kF2Z = 16, kF2X = 64;  // filter output tiles
// Threads per tile of the gather-push-deposit kernel (measured: FP32 runs
// best with 512, FP64, whose LDS footprint is larger, with 256).
#ifndef BFPIC_GPD_THREADS32
#define BFPIC_GPD_THREADS32 512
#endif
#ifndef BFPIC_GPD_THREADS64
#define BFPIC_GPD_THREADS64 256
#endif
template <typename R>
constexpr int kGpdThreads = sizeof(R) == 4 ? BFPIC_GPD_THREADS32 : BFPIC_GPD_THREADS64;
// 3D tiles that gather from global memory (one workgroup per CU by LDS)
#ifndef BFPIC_GPD3_THREADS
#define BFPIC_GPD3_THREADS 512
#endif
constexpr int kGpd3Threads = BFPIC_GPD3_THREADS;
// Row stride along y of their LDS current region (0: its extent).  A wave's
// lanes hold particles of one tile plane, 8 x 8 cells; at the extent's 17
// nodes their FP64 adds share LDS banks, at 22 (the largest stride whose
// 18 x 17 x 22 FP64 region fits the 160 KB) far fewer: 2.94 against 3.13 ms
// per launch at 512 x 128 x 128 (20 nodes: 2.96 ms).
#ifndef BFPIC_GPD3_LDS_Y
#define BFPIC_GPD3_LDS_Y 22
#endif
constexpr int kGpd3LdsY = BFPIC_GPD3_LDS_Y;
// Tiles dispatched largest first (1) or in XCD-aware grid order (0)
#ifndef BFPIC_TILE_ORDER
#define BFPIC_TILE_ORDER 1
#endif
constexpr bool kTileOrder = BFPIC_TILE_ORDER != 0;
// Rows per band of the fused 2D Yee kernel (one wave marches one band)
#ifndef BFPIC_YEE_ROWS
#define BFPIC_YEE_ROWS 16
#endif
constexpr int kYeeRows = BFPIC_YEE_ROWS;
// Tile rows per window of the 2D fold + filter
#ifndef BFPIC_FOLD_ROWS
#define BFPIC_FOLD_ROWS 1
#endif
constexpr int kFoldRows = BFPIC_FOLD_ROWS;
// Rows per thread of the 3D z sweep (fold + z passes)
#ifndef BFPIC_FILT3_ROWS
#define BFPIC_FILT3_ROWS 16
#endif
constexpr int kFilt3Rows = BFPIC_FILT3_ROWS;
constexpr int kF3 = 8;
constexpr int kNumTimers = 7;

static inline int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline int floor_div(int a, int b) { return a >= 0 ? a / b : -((b - 1 - a) / b); }

struct bfpic_ctx {
  bfpic_config cfg;
  hipStream_t stream = nullptr;
  int device = -1;  // HIP device current at create
  std::string err;
  int dim = 2, nz = 0, nx = 0, ny = 1, order = 1;
  bool fp64 = false;
  Geo g{};
  double dt = 0, dz = 0, dx = 0, dy = 1;
  double gamma_b = 1, beta_b = 0, u_b = 0, sb = 0;
  bool inited = false;
  int64_t step = 0, window_cells = 0, next_col = 0;
  bool has_plasma = false;
  int64_t cap = 0, slots_bound = 0, tail_bound = 0;
  DensityK dens{};
  // tiles
  bool tiled = false;
  int TZ = 1, TX = 1, TY = 1, ntx = 1, nty = 1, ntz = 0, ntz_max = 0, zc0 = 0;
  int LZ = 1, LX = 1, LY = 1, LV = 1;
  int64_t maxtiles = 0, maxkeys = 0;
  size_t lds_tiled = 0, lds_limit = 65536;
  bool stage = true;  // tiled kernel stages E, B in LDS (else gathers from global)
  // deterministic mode: currents summed as int64 in units of 1 / fx_scale
  bool det = false;
  double fx_scale = 1.0, fx_inv = 1.0;
  // device buffers
  uint8_t* ws = nullptr;
  int64_t ws_bytes = 0;
  void* F[6] = {};
  void* Fs[6] = {};
  void* Jf[3] = {};
  void* Jo[3] = {};
  void* pid[2] = {};
  void* pxi[2][3] = {};
  void* pdu[2][3] = {};
  void* pw[2] = {};
  int cur = 0;
  int* counts = nullptr;   // [0] slots in use, [1] sorted prefix, [2] slots at last sort,
                           // [4] stragglers listed this step
  int* strag = nullptr;
  int* ovf_rows = nullptr;
  int* tile_start = nullptr;
  int* tile_order = nullptr;
  void* scratch = nullptr;
  unsigned* tbox = nullptr;  // 3D: box word of each tile region
  int* key = nullptr;
  int* rank = nullptr;
  int* perm = nullptr;
  int* cnt = nullptr;
  int* off = nullptr;
  int* bsum = nullptr;
  double* g64a = nullptr;  // FP64 grid scratch (laser potential, rho)
  double* g64b = nullptr;  // FP64 grid scratch (laser Ey, filtered rho)
  double* partials = nullptr;
  double* dout = nullptr;
  int* nanflag = nullptr;
  void* mur_save = nullptr;
  double* wit = nullptr;  // caller's witness state (n x 6), or null
  int nwit = 0;
  int64_t last_sort_nkeys = 0;
  int last_sort_tzmin = 0, last_sort_ntz = 0;
  const int* final_perm = nullptr;  // destination -> source slot of the last sort
  bool have_sort = false;
  // adjoint: taped forward run and reverse sweep
  struct HostCkpt {
    int64_t step, window_cells, next_col, slots_bound, tail_bound;
    int cur;
  };
  double laser_a0 = 0.0;
  bool no_sort = false;      // particle slots stay put (taped runs)
  bool adj_ready = false;    // the tape holds a forward run
  bool adj_recompute = false;
  bool adj_per_direction = false;  // reverse particle step: one dual pass per direction
  bool ant_on = false;             // laser antenna on grid row ant_row
  int ant_row = 0;
  LaserK ant_K{};
  int adj_nsteps = 0, adj_interval = 0;
  int64_t adj_slots = 0;     // slots created by the taped run
  int adj_nwit = 0;          // witnesses bound during the taped run
  bfpic_loss adj_loss{};
  std::vector<HostCkpt> ckpt;
  std::vector<int64_t> adj_wc;  // taped run: window cells at the start of each step
  std::vector<int> adj_shift;   // taped run: window shift at the end of each step
  uint8_t* tape = nullptr;
  int64_t tape_bytes = 0;
  // timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[kNumTimers];
  std::vector<hipEvent_t> pool;
};

#define HIPCHK(h, call)                                                           \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      (h)->err = std::string(#call) + ": " + hipGetErrorString(e_);               \
      return BFPIC_ERR_HIP;                                                       \
    }                                                                             \
  } while (0)

static int fail(bfpic_ctx* h, int code, const std::string& m) {
  if (h) h->err = m;
  return code;
}

// ---------------------------------------------------------------------------
// Timing helpers
// ---------------------------------------------------------------------------
static hipEvent_t take_event(bfpic_ctx* h) {
  if (!h->pool.empty()) {
    hipEvent_t e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
struct Timer {
  bfpic_ctx* h;
  int cls;
  hipEvent_t a = nullptr;
  Timer(bfpic_ctx* h_, int c) : h(h_), cls(c) {
    if (h->timing) {
      a = take_event(h);
      if (a) hipEventRecord(a, h->stream);
    }
  }
  ~Timer() {
    if (h->timing && a) {
      hipEvent_t b = take_event(h);
      if (b) {
        hipEventRecord(b, h->stream);
        h->ev[cls].push_back({a, b});
      }
    }
  }
};

// ---------------------------------------------------------------------------
// Geometry and layout
// ---------------------------------------------------------------------------
static int check_cfg(const bfpic_config* c, std::string& why) {
  if (!c) return (why = "null config", 0);
  if (c->dim != 2 && c->dim != 3) return (why = "dim must be 2 or 3", 0);
  if (c->nz < 4 || c->nx < 2 || (c->dim == 3 && c->ny < 2)) return (why = "grid too small", 0);
  if (!(c->dz > 0 && c->dx > 0 && (c->dim == 2 || c->dy > 0))) return (why = "cell sizes", 0);
  if (!(c->cfl > 0 && c->cfl < 1)) return (why = "cfl must be in (0, 1)", 0);
  if (c->shape_order != 1 && c->shape_order != 2) return (why = "shape_order 1 or 2", 0);
  if (c->filter_passes < 0 || c->filter_passes > 16) return (why = "filter_passes", 0);
  if (c->precision != BFPIC_FP64 && c->precision != BFPIC_FP32_SPLIT) return (why = "precision", 0);
  if (c->z_boundary != BFPIC_BC_PERIODIC && c->z_boundary != BFPIC_BC_MUR) return (why = "z_boundary", 0);
  if (c->ppc < 1) return (why = "ppc", 0);
  if (c->sort_interval < 0) return (why = "sort_interval", 0);
  if (c->gather_form != BFPIC_GATHER_MOMENTUM && c->gather_form != BFPIC_GATHER_ENERGY)
    return (why = "gather_form", 0);
  return 1;
}

template <class TG>
static void set_region(bfpic_ctx* h) {
  h->LZ = TG::LZ;
  h->LX = TG::LX;
  h->LY = TG::LY;
}

// Bytes per element of the tiled kernel's LDS current accumulators, and of
// the tile current scratch and the overflow grid (the working precision, or
// int64 in the deterministic mode).
static size_t acc_bytes(const bfpic_ctx* h) { return h->det || h->fp64 || h->dim == 2 ? 8 : 4; }
static size_t ovf_bytes(const bfpic_ctx* h) { return h->det || h->fp64 ? 8 : 4; }

static void derive(bfpic_ctx* h, const bfpic_config* c) {
  h->cfg = *c;
  h->det = c->deterministic != 0;
  h->dim = c->dim;
  h->nz = c->nz;
  h->nx = c->nx;
  h->ny = c->dim == 3 ? c->ny : 1;
  h->order = c->shape_order;
  h->fp64 = c->precision == BFPIC_FP64;
  h->dz = c->dz;
  h->dx = c->dx;
  h->dy = c->dim == 3 ? c->dy : 1.0;
  h->dt = bfpic_yee_dt(c->dim, c->dz, c->dx, c->dy, c->cfl);
  Geo& g = h->g;
  g.nz = h->nz;
  g.nx = h->nx;
  g.ny = h->ny;
  g.periodic_z = c->z_boundary == BFPIC_BC_PERIODIC;
  g.plane = (int64_t)h->nx * h->ny;
  g.rows = h->nz + 2 * kGuard + 1;
  // tiles
  const int o = h->order;
  if (h->dim == 2) {
    h->TZ = kT2Z;
    h->TX = kT2X;
    h->TY = 1;
    if (o == 1) set_region<TileGeom<2, 1, kT2Z, kT2X, 1, kExc>>(h);
    else set_region<TileGeom<2, 2, kT2Z, kT2X, 1, kExc>>(h);
  } else {
    h->TZ = h->TX = h->TY = kT3;
    if (o == 1) set_region<TileGeom<3, 1, kT3, kT3, kT3, kExc>>(h);
    else set_region<TileGeom<3, 2, kT3, kT3, kT3, kExc>>(h);
  }
  h->LV = h->LZ * h->LX * h->LY;
  // the fold gathers a node from at most three tile regions per axis
  bool fit_x = h->nx % h->TX == 0 && h->LX <= h->nx && h->LX <= 3 * h->TX;
  bool fit_y = h->dim == 2 || (h->ny % h->TY == 0 && h->LY <= h->ny && h->LY <= 3 * h->TY);
  bool fit_z = h->LZ <= 3 * h->TZ &&
               (!g.periodic_z || (h->nz % h->TZ == 0 && h->LZ <= h->nz));
  h->tiled = fit_x && fit_y && fit_z;
  // key tile shape when the LDS path is off: whole transverse planes
  if (!fit_x) h->TX = h->nx;
  if (!fit_y) h->TY = h->ny;
  if (g.periodic_z && h->nz % h->TZ != 0) h->TZ = h->nz;
  h->ntx = h->nx / h->TX;
  h->nty = h->ny / h->TY;
  int lim = o + 1;
  h->ntz_max = g.periodic_z ? h->nz / h->TZ : (int)cdiv(h->nz + 2 * lim + 6, h->TZ) + 2;
  h->maxtiles = (int64_t)h->ntz_max * h->ntx * h->nty;
  h->maxkeys = h->maxtiles * h->TZ * h->TX * h->TY;
  size_t rs = h->fp64 ? 8 : 4;
  // staged E, B in the working precision; currents in FP64 in 2D
  // staged E, B in the working precision; currents in FP64 in 2D, int64 in
  // the deterministic mode
  h->lds_tiled = (size_t)6 * h->LV * rs + (size_t)3 * h->LV * acc_bytes(h);
}

struct Layout {
  int64_t off[64];
  int n = 0;
  int64_t total = 0;
  int64_t add(int64_t bytes) {
    int64_t o = total;
    off[n++] = o;
    total += align256(bytes > 0 ? bytes : 1);
    return o;
  }
};

// Offsets of every buffer inside the workspace (same order in query and create).
static int64_t plan(bfpic_ctx* h, int64_t cap, bfpic_ctx* fill, bfpic_sizes* sz) {
  Layout L;
  const int64_t rs = h->fp64 ? 8 : 4;
  const int64_t grid = h->g.rows * h->g.plane;
  auto P = [&](int64_t bytes) -> void* {
    int64_t o = L.add(bytes);
    return fill ? (void*)(fill->ws + o) : nullptr;
  };
  void* p;
  for (int c = 0; c < 6; c++) {
    p = P(grid * rs);
    if (fill) fill->F[c] = p;
    p = P(grid * rs);
    if (fill) fill->Fs[c] = p;
  }
  for (int c = 0; c < 3; c++) {
    p = P(grid * rs);
    if (fill) fill->Jf[c] = p;
    p = P(grid * (int64_t)ovf_bytes(h));
    if (fill) fill->Jo[c] = p;
  }
  int64_t fields = L.total;
  for (int s = 0; s < 2; s++) {
    p = P(cap * 4);
    if (fill) fill->pid[s] = p;
    for (int a = 0; a < 3; a++) {
      p = P(a < h->dim ? cap * rs : 0);
      if (fill) fill->pxi[s][a] = a < h->dim ? p : nullptr;
    }
    for (int a = 0; a < 3; a++) {
      p = P(cap * rs);
      if (fill) fill->pdu[s][a] = p;
    }
    p = P(cap * rs);
    if (fill) fill->pw[s] = p;
  }
  int64_t parts = L.total - fields;
  p = P(16 * 4);
  if (fill) fill->counts = (int*)p;
  p = P(4 * 4);
  if (fill) fill->ovf_rows = (int*)p;
  p = P((h->maxtiles + 1) * 4);
  if (fill) fill->tile_start = (int*)p;
  p = P(h->maxtiles * 4);
  if (fill) fill->tile_order = (int*)p;
  // tile regions, then one row of tiles that stays zero (read for tile rows
  // outside the co-moving range)
  p = P(h->tiled ? (h->maxtiles + (int64_t)h->ntx * h->nty) * 3 * (int64_t)h->LV *
                       (int64_t)ovf_bytes(h)
                 : 0);
  if (fill) fill->scratch = p;
  p = P(h->tiled && h->dim == 3 ? h->maxtiles * 4 : 0);
  if (fill) fill->tbox = (unsigned*)p;
  p = P(cap * 4);
  if (fill) fill->strag = (int*)p;
  p = P(cap * 4);
  if (fill) fill->key = (int*)p;
  p = P(cap * 4);
  if (fill) fill->rank = (int*)p;
  p = P(cap * 4);
  if (fill) fill->perm = (int*)p;
  p = P((h->maxkeys + 1) * 4);
  if (fill) fill->cnt = (int*)p;
  p = P((h->maxkeys + 1) * 4);
  if (fill) fill->off = (int*)p;
  p = P((cdiv(h->maxkeys + 1, kScanBlock * kScanPer) + 1) * 4);
  if (fill) fill->bsum = (int*)p;
  p = P(grid * 8);
  if (fill) fill->g64a = (double*)p;
  p = P(grid * 8);
  if (fill) fill->g64b = (double*)p;
  p = P(7 * kDiagMaxBlocks * 8);
  if (fill) fill->partials = (double*)p;
  p = P(16 * 8);
  if (fill) fill->dout = (double*)p;
  p = P(4 * 4);
  if (fill) fill->nanflag = (int*)p;
  p = P(4 * h->g.plane * rs);
  if (fill) fill->mur_save = p;
  if (sz) {
    sz->workspace_bytes = L.total;
    sz->field_bytes = fields;
    sz->particle_bytes = parts;
    sz->scratch_bytes = L.total - fields - parts;
  }
  return L.total;
}

// A particle's id is its lattice slot ((k ny + l) nx + j) ppc + s, an int32
// (negative marks a removed slot); columns below kcols fit when
// kcols nx ny ppc <= 2^31.
static bool id_space_fits(const bfpic_ctx* h, int64_t kcols) {
  const int64_t per_col = (int64_t)h->nx * h->ny * h->cfg.ppc;
  return kcols >= 0 && kcols <= (int64_t(1) << 31) / per_col;
}

// ---------------------------------------------------------------------------
// Typed implementation
// ---------------------------------------------------------------------------
template <typename R, int DIM, int ORDER>
struct Impl {
  using TG2 = TileGeom<2, ORDER, kT2Z, kT2X, 1, kExc>;
  using TG3 = TileGeom<3, ORDER, kT3, kT3, kT3, kExc>;
  static constexpr int TZc = DIM == 2 ? kT2Z : kT3;
  static constexpr int TXc = DIM == 2 ? kT2X : kT3;
  static constexpr int TYc = DIM == 2 ? 1 : kT3;

  static PSoA<R> soa(bfpic_ctx* h, int s) {
    PSoA<R> S;
    S.id = (int*)h->pid[s];
    for (int a = 0; a < 3; a++) {
      S.xi[a] = (R*)h->pxi[s][a];
      S.du[a] = (R*)h->pdu[s][a];
    }
    S.w = (R*)h->pw[s];
    return S;
  }
  static Fields<R> fields(bfpic_ctx* h) {
    Fields<R> f;
    for (int c = 0; c < 6; c++) f.F[c] = (R*)h->F[c];
    return f;
  }
  // Granlund-Montgomery magic for division by d (see FastDiv).
  static FastDiv fastdiv(int d) {
    FastDiv f;
    f.d = d;
    if (d <= 1) {
      f.m = 0;
      f.l = 0;
      return f;
    }
    int l = 0;
    while ((1LL << l) < d) l++;
    unsigned __int128 num = ((unsigned __int128)1 << 32) * (((unsigned __int128)1 << l) - d);
    f.m = (uint32_t)(num / (unsigned)d + 1);
    f.l = l;
    return f;
  }
  static LatticeP lattice(bfpic_ctx* h) {
    LatticeP L;
    L.seed = h->cfg.seed;
    L.ppc = h->cfg.ppc;
    L.nx = h->nx;
    L.nyy = h->ny;
    L.load = h->cfg.load;
    L.dppc = fastdiv(h->cfg.ppc);
    L.dnx = fastdiv(h->nx);
    L.dnyy = fastdiv(h->ny);
    return L;
  }
  static Ovf<R> ovf(bfpic_ctx* h) {
    Ovf<R> o;
    for (int c = 0; c < 3; c++) {
      o.J[c] = (R*)h->Jo[c];
      o.Jq[c] = (long long*)h->Jo[c];
    }
    o.rows = h->ovf_rows;
    return o;
  }
  // D = n beta_b dt / dz + window, split into integer and fractional parts.
  static Drift<R> drift(bfpic_ctx* h, int64_t n) {
    double D = (double)n * h->sb + (double)h->window_cells;
    double fl = std::floor(D);
    double fr = D - fl;
    Drift<R> d;
    d.Dint = (int)fl;
    if (sizeof(R) == 4) {
      // quantise to 2^-24 so that birth offset - Dfrac is exact in FP32
      double q = std::nearbyint(fr * 16777216.0) / 16777216.0;
      if (q >= 1.0) {
        q = 0.0;
        d.Dint += 1;
      }
      d.Dfrac = (R)q;
    } else {
      d.Dfrac = (R)fr;
    }
    return d;
  }
  static double drift_cells(bfpic_ctx* h) {
    return (double)h->step * h->sb + (double)h->window_cells;
  }

  static int create_columns(bfpic_ctx* h, int64_t k0, int64_t ncols) {
    int64_t count = ncols * h->nx * h->ny * h->cfg.ppc;
    if (count <= 0) return BFPIC_OK;
    if (!id_space_fits(h, k0 + ncols))
      return fail(h, BFPIC_ERR_CAPACITY, "lattice ids of column " + std::to_string(k0 + ncols) +
                                             " exceed the int32 id space");
    {
      Timer t(h, 5);
      k_create<R><<<(unsigned)cdiv(count, 256), 256, 0, h->stream>>>(
          soa(h, h->cur), lattice(h), h->dens, (int)k0, count, h->counts);
      k_bump_slots<<<1, 1, 0, h->stream>>>(h->counts, (int)count);
    }
    HIPCHK(h, hipGetLastError());
    h->slots_bound += count;
    h->tail_bound += count;
    return BFPIC_OK;
  }

  static int refresh_bound(bfpic_ctx* h) {
    int c[2];
    HIPCHK(h, hipMemcpyAsync(c, h->counts, sizeof(c), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->slots_bound = c[0];
    h->tail_bound = c[0] - c[1];
    return BFPIC_OK;
  }

  // Columns due at the current step: k - D < nz.
  static int64_t due_columns(bfpic_ctx* h) {
    if (!h->has_plasma || h->g.periodic_z) return 0;
    double D = drift_cells(h);
    int64_t k = h->next_col, m = 0;
    while ((double)(k + m) - D < (double)h->nz) m++;
    return m;
  }

  static int inject(bfpic_ctx* h) {
    int64_t m = due_columns(h);
    if (m == 0) return BFPIC_OK;
    int64_t count = m * h->nx * h->ny * h->cfg.ppc;
    if (!id_space_fits(h, h->next_col + m))
      return fail(h, BFPIC_ERR_CAPACITY, "lattice ids of column " + std::to_string(h->next_col + m) +
                                             " exceed the int32 id space");
    if (h->slots_bound + count > h->cap) {
      int rc = refresh_bound(h);
      if (rc) return rc;
      if (h->slots_bound + count > h->cap)
        return fail(h, BFPIC_ERR_CAPACITY,
                    "particle capacity " + std::to_string(h->cap) + " < " +
                        std::to_string(h->slots_bound + count));
    }
    int rc = create_columns(h, h->next_col, m);
    if (rc) return rc;
    h->next_col += m;
    return BFPIC_OK;
  }

  static int sort(bfpic_ctx* h) {
    Timer t(h, 4);
    const Geo& g = h->g;
    int tzmin, ntz;
    if (g.periodic_z) {
      tzmin = 0;
      ntz = h->nz / h->TZ;
    } else {
      double D = drift_cells(h);
      int lim = h->order + 1;
      tzmin = (int)std::floor((D - lim - 2.0) / h->TZ);
      int tzmax = (int)std::floor((D + h->nz + lim + 2.0) / h->TZ);
      ntz = tzmax - tzmin + 1;
      if (ntz > h->ntz_max) return fail(h, BFPIC_ERR_STATE, "tile rows exceed plan");
    }
    SortK K;
    K.TZ = h->TZ;
    K.TX = h->TX;
    K.TY = h->TY;
    K.ntz = ntz;
    K.ntx = h->ntx;
    K.nty = h->nty;
    K.zc0 = tzmin * h->TZ;
    int64_t cpt = (int64_t)h->TZ * h->TX * h->TY;
    int64_t nkeys = (int64_t)ntz * h->ntx * h->nty * cpt;
    K.nkeys = (int)nkeys;
    int64_t nb = std::max<int64_t>(1, cdiv(h->slots_bound, 256));
    PSoA<R> src = soa(h, h->cur), dst = soa(h, 1 - h->cur);
    HIPCHK(h, hipMemsetAsync(h->cnt, 0, (nkeys + 1) * 4, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->counts + 2, h->counts, 4, hipMemcpyDeviceToDevice, h->stream));
    k_sort_keys<R, DIM><<<(unsigned)nb, 256, 0, h->stream>>>(src, lattice(h), g, K, h->counts,
                                                             h->key, h->rank, h->cnt);
    int64_t n = nkeys + 1;
    int64_t nsb = cdiv(n, kScanBlock * kScanPer);
    k_scan_blocks<<<(unsigned)nsb, kScanBlock, 0, h->stream>>>(h->cnt, h->off, h->bsum, n);
    k_scan_sums<<<1, kScanBlock, 0, h->stream>>>(h->bsum, (int)nsb);
    k_scan_add<<<(unsigned)cdiv(n, 256), 256, 0, h->stream>>>(h->off, h->bsum, n);
    k_sort_scatter<<<(unsigned)nb, 256, 0, h->stream>>>(h->counts, h->key, h->rank, h->off,
                                                        h->perm);
    k_sort_cells<<<(unsigned)cdiv(nkeys, 256), 256, 0, h->stream>>>(h->off, src.id, h->perm,
                                                                    (int)nkeys);
    // tiles with at most kInterleaveCells cells are interleaved by rank within
    // cell; the result goes to `rank` (free once the scatter has run)
    const int* fin = h->perm;
    if (cpt <= kInterleaveCells) {
      k_sort_interleave<<<(unsigned)(ntz * h->ntx * h->nty), 256, 0, h->stream>>>(
          h->off, h->perm, h->rank, (int)cpt);
      fin = h->rank;
    }
    h->final_perm = fin;
    k_permute<R><<<(unsigned)nb, 256, 0, h->stream>>>(src, dst, fin, h->off + nkeys);
    int ntiles = ntz * h->ntx * h->nty;
    k_tile_starts<<<(unsigned)cdiv(ntiles + 1, 256), 256, 0, h->stream>>>(
        h->off, h->tile_start, ntiles, (int)cpt, h->counts, (int)nkeys);
    if (kTileOrder && ntiles > 0) {
      // bins of 2^shift particles, the mean tile near bin 32
      int shift = 0;
      while (((int64_t)cpt * h->cfg.ppc >> (shift + 1)) >= 32) shift++;
      k_tile_order<<<1, 1024, 0, h->stream>>>(h->tile_start, ntiles, shift, h->tile_order);
    }
    HIPCHK(h, hipGetLastError());
    h->cur = 1 - h->cur;
    h->ntz = ntz;
    h->zc0 = K.zc0;
    h->tail_bound = 0;
    h->last_sort_nkeys = nkeys;
    h->last_sort_tzmin = tzmin;
    h->last_sort_ntz = ntz;
    h->have_sort = true;
    return BFPIC_OK;
  }

  // Deterministic mode: one fixed-point unit is 2^-e of the current, with e
  // chosen so that a single particle's contribution to a node stays below
  // 2^40 units (int64 sums then hold 2^23 contributions per node).  A
  // contribution is at most 4 max(k) w_max: Esirkepov prefix sums and the
  // pair form are bounded by 3 in shape units, the out-of-plane weight by
  // 13/12 with |v_y| < 1.
  static void set_fixed_scale(bfpic_ctx* h) {
    const DensityK& D = h->dens;
    double nmax = std::fabs(D.n_uniform);
    for (int m = 0; m < D.nknots; m++) nmax = std::max(nmax, std::fabs(D.kn[m]));
    // the channel's largest factor: the box corner, half a box from the axis
    const double rmax2 = D.xa * D.xa + D.ya * D.ya;
    const double wmax = D.gamma_b * nmax * (1.0 + D.ch_k * rmax2) * D.dV_over_ppc;
    double k;
    if (DIM == 2)
      k = std::max({1.0 / (h->dx * h->dt), 1.0 / (h->dz * h->dt), 1.0 / (h->dz * h->dx)});
    else
      k = std::max({1.0 / (h->dx * h->dy * h->dt), 1.0 / (h->dz * h->dy * h->dt),
                    1.0 / (h->dz * h->dx * h->dt)});
    const double bound = 4.0 * k * wmax;
    int e = 0;
    if (bound > 0 && std::isfinite(bound)) e = (int)std::floor(std::log2(std::ldexp(1.0, 40) / bound));
    h->fx_scale = std::ldexp(1.0, e);
    h->fx_inv = std::ldexp(1.0, -e);
  }

  static StepK<R> step_consts(bfpic_ctx* h, bool unscaled = false) {
    StepK<R> P;
    P.g = h->g;
    P.L = lattice(h);
    P.push.ub = (R)h->u_b;
    P.push.gb = (R)h->gamma_b;
    P.push.gb2 = (R)(h->gamma_b * h->gamma_b);
    P.push.qdt2 = (R)(-0.5 * h->dt);
    P.D0 = drift(h, h->step);
    P.D1 = drift(h, h->step + 1);
    P.dtd[0] = (R)(h->dt / h->dz);
    P.dtd[1] = (R)(h->dt / h->dx);
    P.dtd[2] = (R)(h->dt / h->dy);
    if (DIM == 2) {
      P.kj[0] = (R)(1.0 / (h->dx * h->dt));
      P.kj[1] = (R)(1.0 / (h->dz * h->dt));
      P.kj[2] = (R)0;
    } else {
      P.kj[0] = (R)(1.0 / (h->dx * h->dy * h->dt));
      P.kj[1] = (R)(1.0 / (h->dz * h->dy * h->dt));
      P.kj[2] = (R)(1.0 / (h->dz * h->dx * h->dt));
    }
    P.ky2d = (R)(1.0 / (h->dz * h->dx));
    if (h->det && !unscaled) {
      // deterministic mode: the deposit produces fixed-point units directly
      for (int a = 0; a < 3; a++) P.kj[a] = (R)((double)P.kj[a] * h->fx_scale);
      P.ky2d = (R)((double)P.ky2d * h->fx_scale);
    }
    P.galerkin = h->cfg.gather_form == BFPIC_GATHER_ENERGY;
    P.ion_moves = h->sb != 0.0;
    P.remove = !h->g.periodic_z;
    P.lim = ORDER + 1;
    return P;
  }

  // A laser's constants in this context's frame (beta_b of gamma_boost).
  static LaserK laser_consts(bfpic_ctx* h, const bfpic_laser* laser, double gamma_boost) {
    LaserK K;
    K.a0 = laser->a0;
    K.w0 = laser->w0;
    K.L = laser->L;
    K.zc = laser->z_center;
    K.zf = laser->z_focus;
    K.phase = laser->phase;
    K.collimated = laser->collimated;
    K.iz = laser->images_z;
    K.ix = laser->images_x;
    K.iy = laser->images_y;
    K.dim = DIM;
    K.gamma_b = gamma_boost;
    K.gomb = 1.0 / (gamma_boost * (1.0 + h->beta_b));  // gamma (1 - beta)
    K.gbeta = gamma_boost * h->beta_b;
    K.Lz = h->nz * h->dz;
    K.Lx = h->nx * h->dx;
    K.Ly = h->ny * h->dy;
    K.xa = 0.5 * h->nx * h->dx;
    K.ya = DIM == 3 ? 0.5 * h->ny * h->dy : 0.0;
    K.dz = h->dz;
    K.dx = h->dx;
    K.dy = h->dy;
    return K;
  }

  static int set_antenna(bfpic_ctx* h, const bfpic_laser* laser, int row) {
    if (!laser) {
      h->ant_on = false;
      return BFPIC_OK;
    }
    if (!h->inited) return fail(h, BFPIC_ERR_STATE, "init_boosted_plasma first");
    if (row < 1 || row > h->nz - 1) return fail(h, BFPIC_ERR_ARG, "antenna row outside 1 .. nz-1");
    if (!std::isfinite(laser->a0) || !(laser->L >= 0.0) || !(laser->w0 >= 0.0) ||
        laser->images_x < 0 || laser->images_y < 0)
      return fail(h, BFPIC_ERR_ARG, "antenna laser parameters");
    h->ant_K = laser_consts(h, laser, h->gamma_b);
    h->ant_row = row;
    h->ant_on = true;
    return BFPIC_OK;
  }

  // The antenna's current sheet for this step, onto the filtered current.
  static int antenna(bfpic_ctx* h) {
    const double tp = ((double)h->step + 0.5) * h->dt;
    const double zp = ((double)h->ant_row + (double)h->window_cells) * h->dz;
    k_antenna<R><<<(unsigned)cdiv(h->g.plane, 256), 256, 0, h->stream>>>(
        h->g, h->ant_K, tp, zp, h->ant_row, (R*)h->Jf[1]);
    HIPCHK(h, hipGetLastError());
    return BFPIC_OK;
  }

  static FoldK<R> fold_consts(bfpic_ctx* h, const StepK<R>& P) {
    FoldK<R> K;
    K.scratch = h->scratch;
    K.inv_scale = h->fx_inv;
    K.ntz = h->ntz;
    K.ntx = h->ntx;
    K.nty = h->nty;
    K.ntiles = h->tiled ? h->ntz * h->ntx * h->nty : 0;
    // region origin of tile (0,0,0): the same expression as in k_gpd_tiled
    using TG = TileGeom<DIM, ORDER, TZc, TXc, TYc, kExc>;
    K.gz0 = h->zc0 - P.D0.Dint - 1 - kExc - TG::HLO;
    K.gx0 = -kExc - TG::HLO;
    K.gy0 = DIM == 3 ? -kExc - TG::HLO : 0;
    K.TZ = h->TZ;
    K.TX = h->TX;
    K.TY = h->TY;
    K.LZ = h->LZ;
    K.LX = h->LX;
    K.LY = h->LY;
    K.LV = h->LV;
    K.zero_base = h->maxtiles * 3 * (int64_t)h->LV;
    K.box = h->tbox;
    K.o = ovf(h);
    return K;
  }

  static FiltK filt(bfpic_ctx* h) {
    FiltK f;
    f.passes = h->cfg.filter_passes;
    f.comp = h->cfg.filter_compensate ? 1 : 0;
    f.H = f.passes + (f.comp && f.passes > 0 ? 1 : 0);
    double N = (double)f.passes;
    f.a_c = (float)(-0.25 * N);
    f.b_c = (float)(1.0 + 0.5 * N);
    return f;
  }

  // 2D fold + filter on register columns for up to 6 passes per axis; false
  // when the configuration needs the LDS tile kernel instead.
  template <int NP, bool DET>
  static void cols(bfpic_ctx* h, const FoldK<R>& K, const FiltK& fk, const Fields<R>& Jf) {
    using TG = TileGeom<2, ORDER, kT2Z, kT2X, 1, kExc>;
    constexpr int FX = 64 - 2 * NP;
    // windows are rows of tiles: tile row t holds output rows gz0 + t TZ ...,
    // a window kFoldRows of them
    constexpr int WT = kFoldRows;
    const int tz_lo = floor_div(-K.gz0, kT2Z), tz_hi = floor_div(h->nz - K.gz0, kT2Z);
    const int nseg = (tz_hi - tz_lo + WT) / WT, nbx = (int)cdiv(h->nx, FX);
    const int64_t nw = (int64_t)nseg * nbx;
    // FP64 windows run one component per wave (more waves in flight hide the
    // loads); FP32 ones all three (measured faster) unless the grid has too
    // few windows to give every SIMD two waves
    if (sizeof(R) == 8 || nw < 2048)
      k_fold_filter_cols<R, NP, kT2Z, kT2X, TG::LZ, TG::LX, DET, 1, WT>
          <<<dim3((unsigned)cdiv(nw, 4), 3), 256, 0, h->stream>>>(h->g, K, fk, Jf, tz_lo, nseg,
                                                                  nbx, h->ntz_max);
    else
      k_fold_filter_cols<R, NP, kT2Z, kT2X, TG::LZ, TG::LX, DET, 3, WT>
          <<<dim3((unsigned)cdiv(nw, 4), 1), 256, 0, h->stream>>>(h->g, K, fk, Jf, tz_lo, nseg,
                                                                  nbx, h->ntz_max);
  }
  template <bool DET>
  static bool fold_filter_cols(bfpic_ctx* h, const FoldK<R>& K, const FiltK& fk,
                               const Fields<R>& Jf) {
    if constexpr (DIM != 2) {
      return false;
    } else {
      // the column kernel takes at most two tile regions per axis
      if (!h->tiled || h->LX > 2 * h->TX || h->LZ > 2 * h->TZ) return false;
      switch (fk.H) {
        case 0: cols<0, DET>(h, K, fk, Jf); return true;
        case 1: cols<1, DET>(h, K, fk, Jf); return true;
        case 2: cols<2, DET>(h, K, fk, Jf); return true;
        case 3: cols<3, DET>(h, K, fk, Jf); return true;
        case 4: cols<4, DET>(h, K, fk, Jf); return true;
        case 5: cols<5, DET>(h, K, fk, Jf); return true;
        case 6: cols<6, DET>(h, K, fk, Jf); return true;
        default: return false;
      }
    }
  }

  // 3D fold + filter as separable z, x, y sweeps; the window-shift buffers
  // (not state during a step) hold the intermediate grids.
  template <int NP, bool DET>
  static void filt3(bfpic_ctx* h, const FoldK<R>& K, const FiltK& fk, const Fields<R>& Jf) {
    constexpr int SZ = kFilt3Rows, SX = 16, FY = 64 - 2 * NP;
    const Geo& g = h->g;
    Fields<R> T1, T2;
    for (int c = 0; c < 3; c++) {
      T1.F[c] = (R*)h->Fs[c];
      T2.F[c] = (R*)h->Fs[3 + c];
      T1.F[3 + c] = T2.F[3 + c] = nullptr;
    }
    if (!g.periodic_z && h->tiled) {
      // windows aligned to the tile rows' regions (only the regions holding
      // a node are read)
      using TG = TileGeom<3, ORDER, kT3, kT3, kT3, kExc>;
      const int m_first = floor_div(-K.gz0 - NP, kT3);
      const int i0_first = K.gz0 + NP + m_first * kT3;
      const int nsz = (int)cdiv(h->nz + 1 - i0_first, SZ);
      k_filt3_z_aligned<R, NP, SZ, kT3, kT3, kT3, TG::LZ, TG::LX, TG::LY, DET>
          <<<dim3((unsigned)cdiv((int64_t)nsz * g.plane, 256), 1, 3), 256, 0, h->stream>>>(
              g, K, fk, T1, nsz, i0_first, m_first);
    } else {
      const int nsz = (int)cdiv(h->nz + 1, SZ);
      k_filt3_z<R, NP, SZ, kT3, kT3, kT3, DET>
          <<<dim3((unsigned)cdiv((int64_t)nsz * g.plane, 256), 1, 3), 256, 0, h->stream>>>(
              g, K, fk, T1, nsz);
    }
    const int nsx = (int)cdiv(h->nx, SX);
    k_filt3_x<R, NP, SX>
        <<<dim3((unsigned)cdiv((int64_t)(h->nz + 1) * nsx * h->ny, 256), 1, 3), 256, 0,
           h->stream>>>(g, fk, T1, T2, nsx);
    const unsigned nlines = (unsigned)cdiv((int64_t)(h->nz + 1) * h->nx, 4);
    switch (h->ny % 64 == 0 ? h->ny / 64 : 0) {
      case 1:
        k_filt3_y_line<R, NP, 1><<<dim3(nlines, 1, 3), 256, 0, h->stream>>>(g, fk, T2, Jf);
        break;
      case 2:
        k_filt3_y_line<R, NP, 2><<<dim3(nlines, 1, 3), 256, 0, h->stream>>>(g, fk, T2, Jf);
        break;
      case 3:
        k_filt3_y_line<R, NP, 3><<<dim3(nlines, 1, 3), 256, 0, h->stream>>>(g, fk, T2, Jf);
        break;
      case 4:
        k_filt3_y_line<R, NP, 4><<<dim3(nlines, 1, 3), 256, 0, h->stream>>>(g, fk, T2, Jf);
        break;
      default: {
        const int nsy = (int)cdiv(h->ny, FY);
        k_filt3_y<R, NP><<<dim3((unsigned)cdiv((int64_t)(h->nz + 1) * h->nx * nsy, 4), 1, 3),
                           256, 0, h->stream>>>(g, fk, T2, Jf, nsy);
      }
    }
  }
  template <bool DET>
  static bool fold_filter3(bfpic_ctx* h, const FoldK<R>& K, const FiltK& fk,
                           const Fields<R>& Jf) {
    if constexpr (DIM != 3) {
      return false;
    } else {
      switch (fk.H) {
        case 0: filt3<0, DET>(h, K, fk, Jf); return true;
        case 1: filt3<1, DET>(h, K, fk, Jf); return true;
        case 2: filt3<2, DET>(h, K, fk, Jf); return true;
        case 3: filt3<3, DET>(h, K, fk, Jf); return true;
        case 4: filt3<4, DET>(h, K, fk, Jf); return true;
        case 5: filt3<5, DET>(h, K, fk, Jf); return true;
        case 6: filt3<6, DET>(h, K, fk, Jf); return true;
        default: return false;
      }
    }
  }

  template <bool DET>
  static const void* tiled_kernel(bool stage) {
    if constexpr (DIM == 2)
      return (const void*)k_gpd_tiled<R, 2, ORDER, kT2Z, kT2X, 1, kExc, kGpdThreads<R>, DET>;
    else if (stage)
      return (const void*)k_gpd_tiled<R, 3, ORDER, kT3, kT3, kT3, kExc, kGpdThreads<R>, DET>;
    else
      return (const void*)k_gpd_tiled<R, 3, ORDER, kT3, kT3, kT3, kExc, kGpd3Threads, DET,
                                      false, kGpd3LdsY>;
  }

  // Per-configuration kernel set-up at create: opt in to large dynamic LDS.
  static int prepare(bfpic_ctx* h) {
    const int lim = (int)h->lds_limit;
    for (int det = 0; det < 2; det++) {
      const void* fn;
      if (DIM == 2)
        fn = det ? (const void*)k_fold_filter<R, 2, kF2Z, kF2X, 1, kT2Z, kT2X, 1, true>
                 : (const void*)k_fold_filter<R, 2, kF2Z, kF2X, 1, kT2Z, kT2X, 1, false>;
      else
        fn = det ? (const void*)k_fold_filter<R, 3, kF3, kF3, kF3, kT3, kT3, kT3, true>
                 : (const void*)k_fold_filter<R, 3, kF3, kF3, kF3, kT3, kT3, kT3, false>;
      (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    }
    if (h->tiled && h->lds_tiled > 65536) {
      const void* fn = h->det ? tiled_kernel<true>(h->stage) : tiled_kernel<false>(h->stage);
      if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)h->lds_tiled) != hipSuccess)
        h->tiled = false;
    }
    return BFPIC_OK;
  }

  // Gather-push-deposit, current fold and filter; DET selects the
  // fixed-point current sums of the deterministic mode.
  template <bool DET>
  static int particles_and_currents(bfpic_ctx* h, const StepK<R>& P) {
    const Geo& g = h->g;
    Fields<R> F = fields(h);
    PSoA<R> S = soa(h, h->cur);
    Ovf<R> O = ovf(h);
    if (h->tiled && h->ntz > 0) {
      Timer t(h, 0);
      TileK T;
      T.start = h->tile_start;
      // largest first where the fields are staged; the 3D kernel that
      // gathers from global memory keeps the XCD-aware order, whose
      // neighbouring tiles share an L2 (measured 4.9 against 5.8 ms)
      T.order = kTileOrder && (DIM == 2 || h->stage) ? h->tile_order : nullptr;
      T.ntiles = h->ntz * h->ntx * h->nty;
      T.ntx = h->ntx;
      T.nty = h->nty;
      T.zc0 = h->zc0;
      T.strag = h->strag;
      T.nstrag = h->counts + 4;
      T.box = h->tbox;
      if constexpr (DIM == 2)
        k_gpd_tiled<R, 2, ORDER, kT2Z, kT2X, 1, kExc, kGpdThreads<R>, DET>
            <<<T.ntiles, kGpdThreads<R>, h->lds_tiled, h->stream>>>(P, F, S, T, O, h->scratch);
      else if (h->stage)
        k_gpd_tiled<R, 3, ORDER, kT3, kT3, kT3, kExc, kGpdThreads<R>, DET>
            <<<T.ntiles, kGpdThreads<R>, h->lds_tiled, h->stream>>>(P, F, S, T, O, h->scratch);
      else
        k_gpd_tiled<R, 3, ORDER, kT3, kT3, kT3, kExc, kGpd3Threads, DET, false, kGpd3LdsY>
            <<<T.ntiles, kGpd3Threads, h->lds_tiled, h->stream>>>(P, F, S, T, O, h->scratch);
      HIPCHK(h, hipGetLastError());
    }
    {
      // unsorted tail and stragglers (or every slot when not tiled); the
      // straggler count is only known on the device, so the grid strides
      const bool tl = h->tiled && h->ntz > 0;
      int64_t nglob = tl ? h->tail_bound : h->slots_bound;
      unsigned nb = (unsigned)std::min<int64_t>(std::max<int64_t>(cdiv(nglob, 256), tl ? 256 : 1),
                                                 4096);
      if (tl || nglob > 0) {
        Timer t(h, 1);
        k_gpd_global<R, DIM, ORDER, DET><<<nb, 256, 0, h->stream>>>(
            P, F, S, O, h->counts, tl ? 1 : 0, tl ? h->strag : nullptr, h->counts + 4);
        HIPCHK(h, hipGetLastError());
      }
    }
    {
      Timer t(h, 2);
      FoldK<R> K = fold_consts(h, P);
      FiltK fk = filt(h);
      Fields<R> Jf;
      for (int c = 0; c < 3; c++) Jf.F[c] = (R*)h->Jf[c];
      for (int c = 3; c < 6; c++) Jf.F[c] = nullptr;
      if (DIM == 2 && fold_filter_cols<DET>(h, K, fk, Jf)) {
      } else if (DIM == 2) {
        int nbz = (int)cdiv(h->nz + 1, kF2Z), nbx = (int)cdiv(h->nx, kF2X);
        size_t lds = 2 * sizeof(R) * (kF2Z + 2 * fk.H) * (kF2X + 2 * fk.H);
        k_fold_filter<R, 2, kF2Z, kF2X, 1, kT2Z, kT2X, 1, DET>
            <<<nbz * nbx, 256, lds, h->stream>>>(g, K, fk, Jf, nbz, nbx, 1);
      } else if (DIM == 3 && fold_filter3<DET>(h, K, fk, Jf)) {
      } else {
        int nbz = (int)cdiv(h->nz + 1, kF3), nbx = (int)cdiv(h->nx, kF3),
            nby = (int)cdiv(h->ny, kF3);
        size_t lds = 2 * sizeof(R) * (size_t)(kF3 + 2 * fk.H) * (kF3 + 2 * fk.H) * (kF3 + 2 * fk.H);
        k_fold_filter<R, 3, kF3, kF3, kF3, kT3, kT3, kT3, DET>
            <<<nbz * nbx * nby, 256, lds, h->stream>>>(g, K, fk, Jf, nbz, nbx, nby);
      }
      k_ovf_clear<R, DET><<<1024, 256, 0, h->stream>>>(g, O);
      k_ovf_reset<<<1, 1, 0, h->stream>>>(h->ovf_rows, h->counts + 4);
      HIPCHK(h, hipGetLastError());
    }
    if (h->ant_on) {
      const int rc = antenna(h);
      if (rc) return rc;
    }
    return BFPIC_OK;
  }

  // Yee update with Mur at open z ends: B half step, E step, B half step.
  static int yee(bfpic_ctx* h) {
    const Geo& g = h->g;
    if constexpr (DIM == 2) {
      // one fused kernel, E and B double-buffered (F -> Fs, then swapped)
      Timer t(h, 3);
      YeeF<R> Y;
      for (int c = 0; c < 3; c++) {
        Y.E[c] = (const R*)h->F[c];
        Y.B[c] = (const R*)h->F[3 + c];
        Y.J[c] = (const R*)h->Jf[c];
        Y.Eo[c] = (R*)h->Fs[c];
        Y.Bo[c] = (R*)h->Fs[3 + c];
      }
      Y.idz = (R)(1.0 / h->dz);
      Y.idx = (R)(1.0 / h->dx);
      Y.h1 = (R)(0.5 * h->dt);
      Y.h = (R)h->dt;
      Y.mur = (R)((h->dt - h->dz) / (h->dt + h->dz));
      const int nrow = g.periodic_z ? h->nz : h->nz + 1;
      const int tz = kYeeRows;
      const int nband = std::max(1, nrow / tz), nwx = (int)cdiv(h->nx, kYeeCols);
      const int64_t waves = (int64_t)nband * nwx;
      k_yee2d<R><<<(unsigned)cdiv(waves, 4), 256, 0, h->stream>>>(g, Y, nwx, tz, nband);
      HIPCHK(h, hipGetLastError());
      for (int c = 0; c < 6; c++) std::swap(h->F[c], h->Fs[c]);
      return BFPIC_OK;
    }
    {
      Timer t(h, 3);
      YeeK<R> Y;
      for (int c = 0; c < 3; c++) {
        Y.E[c] = (R*)h->F[c];
        Y.B[c] = (R*)h->F[3 + c];
        Y.J[c] = (const R*)h->Jf[c];
      }
      Y.idz = (R)(1.0 / h->dz);
      Y.idx = (R)(1.0 / h->dx);
      Y.idy = (R)(1.0 / h->dy);
      Y.mur = (R)((h->dt - h->dz) / (h->dt + h->dz));
      Y.save = (R*)h->mur_save;
      const unsigned nrow = (unsigned)(g.periodic_z ? h->nz : h->nz + 1);
      const dim3 nb((unsigned)cdiv(g.plane, 256), nrow);
      Y.h = (R)(0.5 * h->dt);
      k_yee_b<R, DIM><<<nb, 256, 0, h->stream>>>(g, Y);
      Y.h = (R)h->dt;
      k_yee_e<R, DIM><<<nb, 256, 0, h->stream>>>(g, Y);
      if (!g.periodic_z) k_mur<R><<<(unsigned)cdiv(g.plane, 256), 256, 0, h->stream>>>(g, Y);
      Y.h = (R)(0.5 * h->dt);
      k_yee_b<R, DIM><<<nb, 256, 0, h->stream>>>(g, Y);
      HIPCHK(h, hipGetLastError());
    }
    return BFPIC_OK;
  }

  static int one_step(bfpic_ctx* h) {
    int rc = inject(h);
    if (rc) return rc;
    bool sort_due = h->cfg.sort_interval > 0 && h->step > 0 && !h->no_sort &&
                    h->step % h->cfg.sort_interval == 0;
    if (sort_due) {
      rc = sort(h);
      if (rc) return rc;
    }
    const Geo& g = h->g;
    StepK<R> P = step_consts(h);
    if (h->nwit > 0) {
      rc = witness_push(h);
      if (rc) return rc;
    }
    rc = h->det ? particles_and_currents<true>(h, P) : particles_and_currents<false>(h, P);
    if (rc) return rc;
    rc = yee(h);
    if (rc) return rc;
    h->step++;
    if (h->cfg.auto_window && !g.periodic_z) {
      double t = (double)h->step * h->dt;
      double due = std::floor((h->cfg.beta_window * t) / h->dz) - (double)h->window_cells;
      if (due != 0.0) {
        rc = shift(h, (int)due);
        if (rc) return rc;
      }
    }
    return BFPIC_OK;
  }

  // ------------------------------------------------------------------------
  // Adjoint.  The caller's tape holds: one checkpoint of the state every
  // `interval` steps (fields E, B; particle slots; device counters), the
  // taped states of one segment (fields and particle state at the start of
  // each step, after its injection), and the adjoint arrays.  Particle slots
  // do not move during a taped run (no re-sort), so a slot is one particle
  // from its injection to its removal.
  // ------------------------------------------------------------------------
  struct Tape {
    uint8_t* ck = nullptr;  // checkpoint 0; checkpoint k at ck + k * ckb
    int64_t ckb = 0;
    uint8_t* sg = nullptr;  // taped step 0 of a segment; step s at sg + s * sgb
    int64_t sgb = 0;
    R* LE[3] = {};
    R* LB[3] = {};
    R* LJf[3] = {};  // adjoint of the filtered current
    R* LJ[3] = {};   // adjoint of the deposited (unfiltered) current
    R* mur = nullptr;
    R* lxi[3] = {};
    R* ldu[3] = {};
    double* lw = nullptr;
    double* wl = nullptr;    // witness adjoints (n x 6)
    double* wfin = nullptr;  // witness states after the last taped step
    int* idb = nullptr;     // birth id of every slot
    double* acc = nullptr;  // [0] loss, [1] <lambda_F, F(0)>, [2..] density gradient
    int64_t total = 0;
  };
  static int64_t gbytes(bfpic_ctx* h) { return h->g.rows * h->g.plane * (int64_t)sizeof(R); }
  static Tape tape_map(bfpic_ctx* h, uint8_t* base, int nsteps, int interval) {
    Tape T;
    const int64_t fb = align256(gbytes(h)), ib = align256(h->cap * 4),
                  rb = align256(h->cap * (int64_t)sizeof(R));
    const int64_t wb = align256(h->nwit * 48);
    // per slot: id, xi (DIM), du (3) and, in a checkpoint, w
    T.ckb = 6 * fb + ib + (DIM + 4) * rb + 256 + wb;
    T.sgb = 6 * fb + ib + (DIM + 3) * rb + 256 + wb;
    const int64_t ncp = cdiv(nsteps, interval);
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
      uint8_t* p = base ? base + o : nullptr;
      o += align256(bytes);
      return p;
    };
    T.ck = take(ncp * T.ckb);
    T.sg = take((int64_t)interval * T.sgb);
    for (int c = 0; c < 3; c++) T.LE[c] = (R*)take(fb);
    for (int c = 0; c < 3; c++) T.LB[c] = (R*)take(fb);
    for (int c = 0; c < 3; c++) T.LJf[c] = (R*)take(fb);
    for (int c = 0; c < 3; c++) T.LJ[c] = (R*)take(fb);
    T.mur = (R*)take(4 * h->g.plane * (int64_t)sizeof(R));
    for (int a = 0; a < DIM; a++) T.lxi[a] = (R*)take(rb);
    for (int a = 0; a < 3; a++) T.ldu[a] = (R*)take(rb);
    T.lw = (double*)take(h->cap * 8);
    T.wl = (double*)take(h->nwit * 48);
    T.wfin = (double*)take(h->nwit * 48);
    T.idb = (int*)take(ib);
    T.acc = (double*)take(8 * (2 + kMaxKnots));
    T.total = o;
    return T;
  }
  // byte offsets inside a checkpoint (ck = true) or a taped step
  static int64_t off_f(bfpic_ctx* h, int c) { return c * align256(gbytes(h)); }
  static int64_t off_id(bfpic_ctx* h) { return 6 * align256(gbytes(h)); }
  static int64_t off_r(bfpic_ctx* h, int k) {  // k: xi (DIM), du0 du1 du2, w
    return off_id(h) + align256(h->cap * 4) + k * align256(h->cap * (int64_t)sizeof(R));
  }
  static int64_t off_tail(bfpic_ctx* h, bool ck) { return off_r(h, ck ? DIM + 4 : DIM + 3); }
  static int64_t off_wit(bfpic_ctx* h, bool ck) { return off_tail(h, ck) + 256; }

  static int copy(bfpic_ctx* h, void* dst, const void* src, int64_t bytes) {
    if (bytes > 0)
      HIPCHK(h, hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDeviceToDevice, h->stream));
    return BFPIC_OK;
  }

  // Copy the state to (save) or from (!save) checkpoint k.
  static int checkpoint(bfpic_ctx* h, const Tape& T, int k, bool save) {
    uint8_t* b = T.ck + (int64_t)k * T.ckb;
    if (!save) {
      const bfpic_ctx::HostCkpt& c = h->ckpt[k];
      h->step = c.step;
      h->window_cells = c.window_cells;
      h->next_col = c.next_col;
      h->slots_bound = c.slots_bound;
      h->tail_bound = c.tail_bound;
      h->cur = c.cur;
    }
    const int64_t n = h->slots_bound, gb = gbytes(h);
    // id, xi (DIM), du (3), w
    void* parts[8];
    int np = 0;
    parts[np++] = h->pid[h->cur];
    for (int a = 0; a < DIM; a++) parts[np++] = h->pxi[h->cur][a];
    for (int a = 0; a < 3; a++) parts[np++] = h->pdu[h->cur][a];
    parts[np++] = h->pw[h->cur];
    int rc = 0;
    for (int c = 0; c < 6 && !rc; c++)
      rc = save ? copy(h, b + off_f(h, c), h->F[c], gb) : copy(h, h->F[c], b + off_f(h, c), gb);
    for (int q = 0; q < np && !rc; q++) {
      uint8_t* t = b + (q == 0 ? off_id(h) : off_r(h, q - 1));
      const int64_t bytes = n * (q == 0 ? 4 : (int64_t)sizeof(R));
      rc = save ? copy(h, t, parts[q], bytes) : copy(h, parts[q], t, bytes);
    }
    if (!rc)
      rc = save ? copy(h, b + off_tail(h, true), h->counts, 16 * 4)
                : copy(h, h->counts, b + off_tail(h, true), 16 * 4);
    if (!rc && h->nwit > 0)
      rc = save ? copy(h, b + off_wit(h, true), h->wit, h->nwit * 48)
                : copy(h, h->wit, b + off_wit(h, true), h->nwit * 48);
    if (rc) return rc;
    if (save) h->ckpt[k] = {h->step, h->window_cells, h->next_col, h->slots_bound, h->tail_bound,
                            h->cur};
    return BFPIC_OK;
  }

  // One step of a taped run; slot >= 0 also stores the state at the start of
  // the step (after injection) as taped step `slot`.
  static int taped_step(bfpic_ctx* h, const Tape& T, int slot) {
    const int64_t s = h->step;
    h->adj_wc[(size_t)s] = h->window_cells;
    int rc = inject(h);
    if (rc) return rc;
    const int64_t n = h->slots_bound;
    if (n > 0)
      k_note_ids<<<(unsigned)cdiv(n, 256), 256, 0, h->stream>>>((const int*)h->pid[h->cur],
                                                                 h->counts, T.idb);
    if (slot >= 0) {
      // the step's tape in one launch: E, B, the particle slots, the slot
      // count and the witnesses
      uint8_t* b = T.sg + (int64_t)slot * T.sgb;
      const int64_t gb = gbytes(h);
      CopyBatch cb;
      int nc = 0;
      auto add = [&](void* dst, const void* src, int64_t bytes) {
        if (bytes <= 0) return;
        cb.dst[nc] = dst;
        cb.src[nc] = src;
        cb.words[nc] = bytes / 4;
        nc++;
      };
      for (int c = 0; c < 6; c++) add(b + off_f(h, c), h->F[c], gb);
      void* parts[7];
      int np = 0;
      parts[np++] = h->pid[h->cur];
      for (int a = 0; a < DIM; a++) parts[np++] = h->pxi[h->cur][a];
      for (int a = 0; a < 3; a++) parts[np++] = h->pdu[h->cur][a];
      for (int q = 0; q < np; q++)
        add(b + (q == 0 ? off_id(h) : off_r(h, q - 1)), parts[q],
            n * (q == 0 ? 4 : (int64_t)sizeof(R)));
      add(b + off_tail(h, false), h->counts, 4);
      if (h->nwit > 0) add(b + off_wit(h, false), h->wit, h->nwit * 48);
      k_copy_batch<<<dim3(256, (unsigned)nc), 256, 0, h->stream>>>(cb);
      HIPCHK(h, hipGetLastError());
    }
    StepK<R> P = step_consts(h);
    if (h->nwit > 0) {
      rc = witness_push(h);
      if (rc) return rc;
    }
    rc = h->det ? particles_and_currents<true>(h, P) : particles_and_currents<false>(h, P);
    if (rc) return rc;
    rc = yee(h);
    if (rc) return rc;
    h->step++;
    // the moving window, as in a plain step; the loss reads the shifted state
    int due = 0;
    if (h->cfg.auto_window && !h->g.periodic_z) {
      const double t = (double)h->step * h->dt;
      due = (int)(std::floor((h->cfg.beta_window * t) / h->dz) - (double)h->window_cells);
      if (due != 0) {
        rc = shift(h, due);
        if (rc) return rc;
      }
    }
    h->adj_shift[(size_t)s] = due;
    const bfpic_loss& L = h->adj_loss;
    if (!h->adj_recompute && h->step >= L.step_first && h->step <= L.step_last) {
      const int nb = (L.i1 - L.i0 + 1) * (L.j1 - L.j0 + 1) * (L.k1 - L.k0 + 1);
      const double sc = 1.0 / ((double)(L.step_last - L.step_first + 1) * nb);
      k_loss_ez<R><<<(unsigned)std::min<int64_t>(cdiv(nb, 256), 256), 256, 0, h->stream>>>(
          h->g, (const R*)h->F[2], L.i0, L.i1, L.j0, L.j1, L.k0, L.k1, sc, T.acc);
      HIPCHK(h, hipGetLastError());
    }
    return BFPIC_OK;
  }

  static int adjoint_check(bfpic_ctx* h, int nsteps, int interval) {
    if (!h->inited) return fail(h, BFPIC_ERR_STATE, "init_boosted_plasma first");
    if (h->ant_on) return fail(h, BFPIC_ERR_UNSUPPORTED, "the adjoint is built without antenna");
    if (nsteps < 1 || interval < 1) return fail(h, BFPIC_ERR_ARG, "nsteps, interval >= 1");
    return BFPIC_OK;
  }

  static int forward_loss(bfpic_ctx* h, int nsteps, int interval, const bfpic_loss* L,
                          void* tape, int64_t tape_bytes, double* out) {
    int rc = adjoint_check(h, nsteps, interval);
    if (rc) return rc;
    if (h->step != 0) return fail(h, BFPIC_ERR_STATE, "a taped run starts right after init");
    const int rz = h->g.periodic_z ? h->nz - 1 : h->nz - 1;
    if (L->step_first < 1 || L->step_last > nsteps || L->step_first > L->step_last ||
        L->i0 < 0 || L->i1 > rz || L->i0 > L->i1 || L->j0 < 0 || L->j1 >= h->nx || L->j0 > L->j1)
      return fail(h, BFPIC_ERR_ARG, "loss window or box out of range");
    if (DIM == 3 ? (L->k0 < 0 || L->k1 >= h->ny || L->k0 > L->k1) : (L->k0 != 0 || L->k1 != 0))
      return fail(h, BFPIC_ERR_ARG, "loss box y range out of range (2D: k0 = k1 = 0)");
    if (!std::isfinite(L->witness_weight) || (L->witness_weight != 0.0 && h->nwit == 0))
      return fail(h, BFPIC_ERR_ARG, "witness weight needs bound witnesses");
    Tape T = tape_map(h, (uint8_t*)tape, nsteps, interval);
    if (!tape || tape_bytes < T.total || ((uintptr_t)tape & 255))
      return fail(h, BFPIC_ERR_ARG, "tape too small or misaligned");
    h->tape = (uint8_t*)tape;
    h->tape_bytes = tape_bytes;
    h->adj_nsteps = nsteps;
    h->adj_interval = interval;
    h->adj_loss = *L;
    h->adj_ready = false;
    h->adj_recompute = false;
    h->no_sort = true;
    h->ckpt.assign((size_t)cdiv(nsteps, interval), bfpic_ctx::HostCkpt{});
    h->adj_wc.assign((size_t)nsteps, 0);
    h->adj_shift.assign((size_t)nsteps, 0);
    HIPCHK(h, hipMemsetAsync(T.acc, 0, 8 * (2 + kMaxKnots), h->stream));
    HIPCHK(h, hipMemsetAsync(T.idb, 0xff, (size_t)h->cap * 4, h->stream));
    for (int s = 0; s < nsteps; s++) {
      if (s % interval == 0) {
        rc = checkpoint(h, T, s / interval, true);
        if (rc) return rc;
      }
      rc = taped_step(h, T, -1);
      if (rc) return rc;
    }
    h->adj_slots = h->slots_bound;
    h->adj_nwit = h->nwit;
    if (h->nwit > 0) {
      rc = copy(h, T.wfin, h->wit, h->nwit * 48);
      if (rc) return rc;
      if (L->witness_weight != 0.0) {
        k_witness_energy<<<(unsigned)cdiv(h->nwit, 256), 256, 0, h->stream>>>(
            h->wit, h->nwit, L->witness_weight / h->nwit, h->gamma_b, h->beta_b, T.acc);
        HIPCHK(h, hipGetLastError());
      }
    }
    double v = 0.0;
    HIPCHK(h, hipMemcpyAsync(&v, T.acc, 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    *out = v;
    h->adj_ready = true;
    return BFPIC_OK;
  }

  static int adjoint(bfpic_ctx* h, double* da0, double* dn, int nn) {
    {
      if (!h->adj_ready) return fail(h, BFPIC_ERR_STATE, "no taped forward run");
      if (DIM == 3 && h->adj_per_direction)
        return fail(h, BFPIC_ERR_UNSUPPORTED, "the per-direction reference is built for 2D runs");
      if (h->nwit != h->adj_nwit)
        return fail(h, BFPIC_ERR_STATE, "witnesses rebound since the taped run");
      const int nk = h->dens.nknots >= 2 ? h->dens.nknots : 1;
      if (nn < nk) return fail(h, BFPIC_ERR_ARG, "density gradient needs one value per knot");
      const int nsteps = h->adj_nsteps, interval = h->adj_interval;
      Tape T = tape_map(h, h->tape, nsteps, interval);
      const Geo& g = h->g;
      const int64_t gb = gbytes(h);
      for (int c = 0; c < 3; c++) {
        HIPCHK(h, hipMemsetAsync(T.LE[c], 0, gb, h->stream));
        HIPCHK(h, hipMemsetAsync(T.LB[c], 0, gb, h->stream));
        HIPCHK(h, hipMemsetAsync(T.LJf[c], 0, gb, h->stream));
        HIPCHK(h, hipMemsetAsync(T.LJ[c], 0, gb, h->stream));
      }
      const int64_t rb = h->cap * (int64_t)sizeof(R);
      for (int a = 0; a < DIM; a++) HIPCHK(h, hipMemsetAsync(T.lxi[a], 0, rb, h->stream));
      for (int a = 0; a < 3; a++) HIPCHK(h, hipMemsetAsync(T.ldu[a], 0, rb, h->stream));
      HIPCHK(h, hipMemsetAsync(T.lw, 0, h->cap * 8, h->stream));
      const bfpic_loss& L = h->adj_loss;
      const int nbox = (L.i1 - L.i0 + 1) * (L.j1 - L.j0 + 1) * (L.k1 - L.k0 + 1);
      const R lsc = (R)(1.0 / ((double)(L.step_last - L.step_first + 1) * nbox));
      AdjYeeK<R> Y;
      for (int c = 0; c < 3; c++) {
        Y.LE[c] = T.LE[c];
        Y.LB[c] = T.LB[c];
        Y.LJ[c] = T.LJf[c];
      }
      Y.idz = (R)(1.0 / h->dz);
      Y.idx = (R)(1.0 / h->dx);
      Y.idy = (R)(DIM == 3 ? 1.0 / h->dy : 0.0);
      const R mur = (R)((h->dt - h->dz) / (h->dt + h->dz));
      const int64_t nrow = g.periodic_z ? h->nz : h->nz + 1;
      const unsigned nbg = (unsigned)cdiv(nrow * g.plane, 256);
      const unsigned nbs = (unsigned)cdiv(g.rows * g.plane, 256);
      const unsigned nbp = (unsigned)cdiv(g.plane, 256);
      FiltK fk = filt(h);
      // filter transpose tiles: 2D kF2Z x kF2X, 3D kF3 cubes
      const int fnbz = (int)cdiv(h->nz + 1, DIM == 2 ? kF2Z : kF3);
      const int fnbx = (int)cdiv(h->nx, DIM == 2 ? kF2X : kF3);
      const int fnby = DIM == 2 ? 1 : (int)cdiv(h->ny, kF3);
      const size_t flds = DIM == 2 ? 2 * sizeof(R) * (kF2Z + 2 * fk.H) * (kF2X + 2 * fk.H)
                                   : 2 * sizeof(R) * (size_t)(kF3 + 2 * fk.H) *
                                         (kF3 + 2 * fk.H) * (kF3 + 2 * fk.H);
      Fields<R> LJ, LF;
      for (int c = 0; c < 3; c++) {
        LJ.F[c] = T.LJ[c];
        LF.F[c] = T.LE[c];
        LF.F[3 + c] = T.LB[c];
        LJ.F[3 + c] = nullptr;
      }
      Grid3R<R> fio;
      for (int c = 0; c < 3; c++) {
        fio.in[c] = T.LJf[c];
        fio.out[c] = T.LJ[c];
      }
      AdjSlots<R> A;
      for (int a = 0; a < 3; a++) A.lxi[a] = a < DIM ? T.lxi[a] : nullptr;
      for (int a = 0; a < 3; a++) A.ldu[a] = T.ldu[a];
      A.lw = T.lw;
      const bool wit_adj = h->nwit > 0 && L.witness_weight != 0.0;
      const unsigned nbw = (unsigned)cdiv(std::max(h->nwit, 1), 256);
      if (wit_adj) {
        k_witness_energy_seed<<<nbw, 256, 0, h->stream>>>(
            T.wfin, h->nwit, L.witness_weight / h->nwit, h->gamma_b, h->beta_b, T.wl);
        HIPCHK(h, hipGetLastError());
      }
      const int ncp = (int)cdiv(nsteps, interval);
      for (int k = ncp - 1; k >= 0; k--) {
        const int s0 = k * interval, s1 = std::min(nsteps, s0 + interval);
        int rc = checkpoint(h, T, k, false);
        if (rc) return rc;
        h->adj_recompute = true;
        for (int s = s0; s < s1; s++) {
          rc = taped_step(h, T, s - s0);
          if (rc) return rc;
        }
        for (int s = s1 - 1; s >= s0; s--) {
          if (s + 1 >= L.step_first && s + 1 <= L.step_last)
            k_loss_ez_adj<R><<<(unsigned)cdiv(nbox, 256), 256, 0, h->stream>>>(
                g, T.LE[2], L.i0, L.i1, L.j0, L.j1, L.k0, L.k1, lsc);
          // transpose of the window shift that ended step s: lambda moves back
          // by the shift, through the current-adjoint arrays (free here: the
          // step's Yee transpose rewrites them) and one batched copy
          if (const int sh = h->adj_shift[(size_t)s]) {
            ShiftAdj<R> S6;
            for (int c = 0; c < 3; c++) {
              S6.src[c] = T.LE[c];
              S6.src[3 + c] = T.LB[c];
              S6.dst[c] = T.LJf[c];
              S6.dst[3 + c] = T.LJ[c];
            }
            k_shift_adj<R><<<dim3(nbs, 6), 256, 0, h->stream>>>(g, S6, sh);
            CopyBatch cb;
            for (int c = 0; c < 3; c++) {
              cb.src[c] = T.LJf[c];
              cb.dst[c] = T.LE[c];
              cb.src[3 + c] = T.LJ[c];
              cb.dst[3 + c] = T.LB[c];
            }
            for (int c = 0; c < 6; c++) cb.words[c] = gb / 4;
            k_copy_batch<<<dim3(256, 6), 256, 0, h->stream>>>(cb);
          }
          Y.h = (R)(0.5 * h->dt);
          k_adj_yee_b<R, DIM><<<nbg, 256, 0, h->stream>>>(g, Y);
          if (!g.periodic_z) k_adj_mur_pre<R><<<nbp, 256, 0, h->stream>>>(g, Y, mur, T.mur);
          Y.h = (R)h->dt;
          k_adj_yee_e<R, DIM><<<nbg, 256, 0, h->stream>>>(g, Y);
          if (!g.periodic_z) k_adj_mur_post<R><<<nbp, 256, 0, h->stream>>>(g, Y, T.mur);
          Y.h = (R)(0.5 * h->dt);
          k_adj_yee_b<R, DIM><<<nbg, 256, 0, h->stream>>>(g, Y);
          if constexpr (DIM == 2)
            k_filter_grid_r3<R, kF2Z, kF2X>
                <<<dim3((unsigned)(fnbz * fnbx), 3), 256, flds, h->stream>>>(g, fk, fio, fnbz,
                                                                             fnbx);
          else
            k_filter_grid_r3d<R, kF3><<<dim3((unsigned)(fnbz * fnbx * fnby), 3), 256, flds,
                                        h->stream>>>(g, fk, fio, fnbz, fnbx, fnby);
          // particles of step s
          uint8_t* b = T.sg + (int64_t)(s - s0) * T.sgb;
          const int64_t save_step = h->step, save_wc = h->window_cells;
          h->step = s;
          h->window_cells = h->adj_wc[(size_t)s];
          StepK<R> P = step_consts(h, true);
          h->step = save_step;
          h->window_cells = save_wc;
          Fields<R> F;
          for (int c = 0; c < 6; c++) F.F[c] = (R*)(b + off_f(h, c));
          TapeParticles<R> TP;
          TP.id = (const int*)(b + off_id(h));
          for (int a = 0; a < 3; a++) TP.xi[a] = a < DIM ? (const R*)(b + off_r(h, a)) : nullptr;
          for (int a = 0; a < 3; a++) TP.du[a] = (const R*)(b + off_r(h, DIM + a));
          TP.w = (const R*)h->pw[h->cur];
          TP.count = (const int*)(b + off_tail(h, false));
          const unsigned nbq = (unsigned)std::max<int64_t>(1, std::min<int64_t>(
                                   cdiv(std::max<int64_t>(h->slots_bound, 1), 256), 4096));
          if constexpr (DIM == 2) {
            if (h->adj_per_direction)
              k_adj_particles<R, ORDER><<<nbq, 256, 0, h->stream>>>(P, F, TP, LJ, LF, A);
            else
              k_adj_particles_staged<R, ORDER, 2><<<nbq, 256, 0, h->stream>>>(P, F, TP, LJ, LF,
                                                                               A);
            if (wit_adj) {
              WitK W{(double*)(b + off_wit(h, false)), h->nwit,
                     {h->dt / h->dz, h->dt / h->dx, h->dt / h->dy}, -0.5 * h->dt,
                     h->cfg.gather_form};
              k_adj_witness<R, ORDER><<<nbw, 256, 0, h->stream>>>(g, F, W, T.wl, LF);
            }
          } else {
            k_adj_particles_staged<R, ORDER, 3><<<nbq, 256, 0, h->stream>>>(P, F, TP, LJ, LF, A);
            if (wit_adj) {
              WitK W{(double*)(b + off_wit(h, false)), h->nwit,
                     {h->dt / h->dz, h->dt / h->dx, h->dt / h->dy}, -0.5 * h->dt,
                     h->cfg.gather_form};
              k_adj_witness<R, ORDER, 3><<<nbw, 256, 0, h->stream>>>(g, F, W, T.wl, LF);
            }
          }
          HIPCHK(h, hipGetLastError());
        }
      }
      h->adj_recompute = false;
      // parameter gradients
      HIPCHK(h, hipMemsetAsync(T.acc + 1, 0, 8 * (1 + kMaxKnots), h->stream));
      for (int c = 0; c < 6; c++) {
        const R* lam = c < 3 ? T.LE[c] : T.LB[c - 3];
        k_dot_fields<R><<<256, 256, 0, h->stream>>>(lam, (const R*)(T.ck + off_f(h, c)),
                                                   g.rows * g.plane, T.acc + 1);
      }
      // every slot the forward run created
      const int64_t nslots = h->adj_slots;
      k_knot_grad<<<256, 256, 0, h->stream>>>(T.idb, T.lw, nslots, lattice(h), h->dens, T.acc + 2);
      HIPCHK(h, hipGetLastError());
      double host[2 + kMaxKnots];
      HIPCHK(h, hipMemcpyAsync(host, T.acc, sizeof(host), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      *da0 = h->laser_a0 != 0.0 ? host[1] / h->laser_a0 : 0.0;
      for (int m = 0; m < nk; m++) dn[m] = host[2 + m];
      return BFPIC_OK;
    }
  }

  static int steps(bfpic_ctx* h, int n) {
    for (int s = 0; s < n; s++) {
      int rc = one_step(h);
      if (rc) return rc;
    }
    return BFPIC_OK;
  }

  static int shift(bfpic_ctx* h, int n) {
    if (n == 0) return BFPIC_OK;
    Timer t(h, 6);
    unsigned nb = (unsigned)cdiv(h->g.rows * h->g.plane, 256);
    for (int c = 0; c < 6; c++) {
      int half = c == 2 || c == 3 || c == 4;
      k_shift<R><<<nb, 256, 0, h->stream>>>(h->g, (const R*)h->F[c], (R*)h->Fs[c], n, half);
      std::swap(h->F[c], h->Fs[c]);
    }
    if (h->nwit > 0)
      k_witness_shift<<<(unsigned)cdiv(h->nwit, 256), 256, 0, h->stream>>>(h->wit, h->nwit, n);
    HIPCHK(h, hipGetLastError());
    h->window_cells += n;
    return BFPIC_OK;
  }

  // Witness electrons through the start-of-step fields (FP64).
  static int witness_push(bfpic_ctx* h) {
    WitK W{h->wit, h->nwit, {h->dt / h->dz, h->dt / h->dx, h->dt / h->dy}, -0.5 * h->dt,
           h->cfg.gather_form};
    k_witness_push<R, DIM, ORDER><<<(unsigned)cdiv(h->nwit, 256), 256, 0, h->stream>>>(
        h->g, fields(h), W);
    HIPCHK(h, hipGetLastError());
    return BFPIC_OK;
  }

  // Zeroes every device buffer a step expects to find zeroed or reset: the
  // fields and the shift buffers, the filtered current, the whole overflow
  // grid, the counters, the row of zero tiles the fold reads past the last
  // tile, and the overflow row range.
  static int reset_device(bfpic_ctx* h) {
    const Geo& g = h->g;
    const int64_t rs = h->fp64 ? 8 : 4;
    const int64_t grid = g.rows * g.plane;
    for (int c = 0; c < 6; c++) {
      HIPCHK(h, hipMemsetAsync(h->F[c], 0, grid * rs, h->stream));
      HIPCHK(h, hipMemsetAsync(h->Fs[c], 0, grid * rs, h->stream));
    }
    for (int c = 0; c < 3; c++) {
      HIPCHK(h, hipMemsetAsync(h->Jf[c], 0, grid * rs, h->stream));
      HIPCHK(h, hipMemsetAsync(h->Jo[c], 0, grid * (int64_t)ovf_bytes(h), h->stream));
    }
    HIPCHK(h, hipMemsetAsync(h->counts, 0, 16 * 4, h->stream));
    if (h->tiled) {
      const int64_t tile_bytes = 3 * (int64_t)h->LV * (int64_t)ovf_bytes(h);
      HIPCHK(h, hipMemsetAsync((char*)h->scratch + h->maxtiles * tile_bytes, 0,
                               (int64_t)h->ntx * h->nty * tile_bytes, h->stream));
    }
    k_ovf_reset<<<1, 1, 0, h->stream>>>(h->ovf_rows, h->counts + 4);
    HIPCHK(h, hipGetLastError());
    return BFPIC_OK;
  }

  // Every check init makes, before it changes any host or device state.
  static int init_args(bfpic_ctx* h, const bfpic_density* d) {
    if (!d) return BFPIC_OK;
    if (d->nknots >= 2) {
      if (d->nknots > kMaxKnots) return fail(h, BFPIC_ERR_ARG, "at most 32 density knots");
      if (!d->z_lab || !d->n) return fail(h, BFPIC_ERR_ARG, "density knots: null array");
      for (int m = 0; m + 1 < d->nknots; m++)
        if (!(d->z_lab[m + 1] > d->z_lab[m]))
          return fail(h, BFPIC_ERR_ARG, "density knots: z_lab must increase");
    }
    if (!(d->channel_depth >= 0.0) || !std::isfinite(d->channel_depth) ||
        (d->channel_depth > 0.0 && !(d->channel_radius > 0.0)))
      return fail(h, BFPIC_ERR_ARG, "channel: depth >= 0, radius > 0");
    const int64_t count = (int64_t)h->nz * h->nx * h->ny * h->cfg.ppc;
    if (count > h->cap)
      return fail(h, BFPIC_ERR_CAPACITY, "initial particles " + std::to_string(count) +
                                             " exceed capacity " + std::to_string(h->cap));
    if (!id_space_fits(h, h->nz))
      return fail(h, BFPIC_ERR_CAPACITY, "initial lattice ids exceed the int32 id space");
    return BFPIC_OK;
  }

  static int init(bfpic_ctx* h, double gamma_boost, const bfpic_density* d,
                  const bfpic_laser* laser) {
    const Geo& g = h->g;
    int rca = init_args(h, d);
    if (rca) return rca;
    // from here on a failure leaves the context needing a new init
    h->inited = false;
    h->ant_on = false;  // init removes the antenna (its constants depend on the boost)
    h->gamma_b = gamma_boost;
    h->beta_b = bfpic_beta(gamma_boost);
    h->u_b = bfpic_drift_u(gamma_boost);
    h->sb = (h->beta_b * h->dt) / h->dz;
    h->step = 0;
    h->window_cells = 0;
    h->next_col = 0;
    h->has_plasma = d != nullptr;
    h->laser_a0 = laser ? laser->a0 : 0.0;
    h->adj_ready = false;
    h->no_sort = false;
    h->wit = nullptr;
    h->nwit = 0;
    h->slots_bound = 0;
    h->tail_bound = 0;
    h->have_sort = false;
    int rc0 = reset_device(h);
    if (rc0) return rc0;
    const int64_t grid = g.rows * g.plane;
    if (laser) {
      const LaserK K = laser_consts(h, laser, gamma_boost);
      HIPCHK(h, hipMemsetAsync(h->g64a, 0, grid * 8, h->stream));
      HIPCHK(h, hipMemsetAsync(h->g64b, 0, grid * 8, h->stream));
      int64_t nrow = g.periodic_z ? h->nz : h->nz + 1;
      unsigned nb = (unsigned)cdiv(nrow * g.plane, 256);
      k_laser_a<R><<<nb, 256, 0, h->stream>>>(g, K, (R*)h->F[1], h->g64a, h->g64b);
      k_laser_b<R><<<nb, 256, 0, h->stream>>>(g, h->g64a, h->dz, h->dx, (R*)h->F[3], (R*)h->F[5]);
      if (DIM == 3)
        k_laser_ez<R><<<(unsigned)cdiv(g.plane, 256), 256, 0, h->stream>>>(g, h->g64b, h->dz,
                                                                         h->dy, (R*)h->F[2]);
      HIPCHK(h, hipGetLastError());
    }
    if (d) {
      DensityK& D = h->dens;
      D.n_uniform = d->n_uniform;
      D.nknots = d->nknots >= 2 ? d->nknots : 0;
      for (int m = 0; m < D.nknots; m++) {
        D.kz[m] = d->z_lab[m];
        D.kn[m] = d->n[m];
      }
      D.gamma_b = gamma_boost;
      D.dz = h->dz;
      D.dV_over_ppc = h->dz * h->dx * (DIM == 3 ? h->dy : 1.0) / h->cfg.ppc;
      for (int a = 0; a < 3; a++) D.du0[a] = d->du[a];
      D.ch_k = d->channel_depth > 0.0
                   ? d->channel_depth / (d->channel_radius * d->channel_radius) : 0.0;
      D.dx = h->dx;
      D.dy = h->dy;
      D.xa = 0.5 * h->nx * h->dx;
      D.ya = DIM == 3 ? 0.5 * h->ny * h->dy : 0.0;
      D.dim3 = DIM == 3;
      set_fixed_scale(h);
      int rc = create_columns(h, 0, h->nz);
      if (rc) return rc;
      h->next_col = h->nz;
      rc = sort(h);
      if (rc) return rc;
    }
    h->inited = true;
    return BFPIC_OK;
  }

  // Reduction buffers of the diagnostics: block partials of the field sums
  // (2 per block), particle sums (4 per block) and Gauss maxima (1 per
  // block), the final values and the non-finite flag.
  struct DiagBufs {
    double *pf, *pp, *pg, *dout;
    int* nanflag;
  };
  // Blocks per reduction: one per 2048 items, at most kDiagMaxBlocks.
  static int diag_blocks(int64_t items) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(kDiagMaxBlocks, cdiv(items, 2048)));
  }

  static int diag(bfpic_ctx* h, bfpic_diag* o, double* lineout) {
    DiagBufs B{h->partials, h->partials + 2 * kDiagMaxBlocks, h->partials + 6 * kDiagMaxBlocks,
               h->dout, h->nanflag};
    return diag_with(h, o, lineout, B);
  }

  // The same diagnostics with every reduction buffer in the static scratch
  // at `base` (device address of `scratch` on the context's device).
  static int diag_static(bfpic_ctx* h, bfpic_diag* o, double* lineout, uint8_t* base) {
    DiagBufs B;
    B.nanflag = (int*)base;
    B.dout = (double*)(base + 256);
    B.pf = B.dout + 16;
    B.pp = B.pf + 2 * kDiagMaxBlocks;
    B.pg = B.pp + 4 * kDiagMaxBlocks;
    const int64_t need = (int64_t)((uint8_t*)(B.pg + kDiagMaxBlocks) - base);
    if (need > kStaticScratchBytes)
      return fail(h, BFPIC_ERR_ARG, "diagnostics need " + std::to_string(need) +
                                        " bytes of static scratch, above its " +
                                        std::to_string(kStaticScratchBytes));
    return diag_with(h, o, lineout, B);
  }

  static int diag_with(bfpic_ctx* h, bfpic_diag* o, double* lineout, const DiagBufs& B) {
    const Geo& g = h->g;
    Fields<R> F = fields(h);
    PSoA<R> S = soa(h, h->cur);
    double* pf = B.pf;
    double* pp = B.pp;
    double* pg = B.pg;
    const int64_t grid = g.rows * g.plane;
    // cleared by fill kernels, so that no memset node enters a captured graph
    k_zero_f64<<<1, 64, 0, h->stream>>>((double*)B.nanflag, 1);
    k_zero_f64<<<(unsigned)std::min<int64_t>(cdiv(grid, 256), 4096), 256, 0, h->stream>>>(
        h->g64a, grid);
    k_zero_f64<<<(unsigned)std::min<int64_t>(cdiv(grid, 256), 4096), 256, 0, h->stream>>>(
        h->g64b, grid);
    const int nbf = diag_blocks((int64_t)(h->nz + 1) * g.plane);
    const int nbp = diag_blocks(h->slots_bound);
    const int nbg = diag_blocks((int64_t)(h->nz + 1) * g.plane);
    k_diag_fields<R><<<nbf, kDiagBlock, 0, h->stream>>>(g, F, pf, B.nanflag);
    k_diag_particles<R, DIM><<<nbp, kDiagBlock, 0, h->stream>>>(S, h->counts, h->u_b, h->gamma_b,
                                                                pp, B.nanflag);
    double dV = h->dz * h->dx * (DIM == 3 ? h->dy : 1.0);
    if (h->slots_bound > 0)
      k_rho<R, DIM, ORDER><<<(unsigned)cdiv(h->slots_bound, 256), 256, 0, h->stream>>>(
          S, lattice(h), drift(h, h->step), g, h->counts, 1.0 / dV, h->g64a);
    FiltK fk = filt(h);
    if (DIM == 2) {
      int nbz = (int)cdiv(h->nz + 1, kF2Z), nbx = (int)cdiv(h->nx, kF2X);
      size_t lds = 2 * 8 * (size_t)(kF2Z + 2 * fk.H) * (kF2X + 2 * fk.H);
      k_filter_grid<2, kF2Z, kF2X, 1><<<nbz * nbx, 256, lds, h->stream>>>(g, fk, h->g64a,
                                                                          h->g64b, nbz, nbx, 1);
    } else {
      int nbz = (int)cdiv(h->nz + 1, kF3), nbx = (int)cdiv(h->nx, kF3), nby = (int)cdiv(h->ny, kF3);
      size_t lds = 2 * 8 * (size_t)(kF3 + 2 * fk.H) * (kF3 + 2 * fk.H) * (kF3 + 2 * fk.H);
      k_filter_grid<3, kF3, kF3, kF3><<<nbz * nbx * nby, 256, lds, h->stream>>>(
          g, fk, h->g64a, h->g64b, nbz, nbx, nby);
    }
    int lo, hi;
    if (g.periodic_z) {
      lo = 0;
      hi = h->nz - 1;
    } else {
      int b = h->cfg.filter_passes + h->order + 4;
      lo = b;
      hi = h->nz - b;
    }
    if (hi >= lo)
      k_gauss<R, DIM><<<nbg, kDiagBlock, 0, h->stream>>>(g, F, h->g64b, 1.0 / h->dz, 1.0 / h->dx,
                                                         1.0 / h->dy, lo, hi, pg);
    else
      k_zero_f64<<<1, 256, 0, h->stream>>>(pg, nbg);
    k_diag_final<R><<<1, kDiagBlock, 0, h->stream>>>(g, (const R*)h->F[2], pf, nbf, pp, nbp, pg,
                                                     nbg, B.dout, lineout);
    HIPCHK(h, hipGetLastError());
    double out[8];
    int nanf = 0;
    HIPCHK(h, hipMemcpyAsync(out, B.dout, sizeof(out), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(&nanf, B.nanflag, 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    o->step = h->step;
    o->t = (double)h->step * h->dt;
    o->window_cells = (double)h->window_cells;
    o->drift_cells = drift_cells(h);
    o->ue = 0.5 * out[0] * dV;
    o->ub = 0.5 * out[1] * dV;
    o->ukin = out[2];
    o->ukin_drift = out[3];
    o->charge = out[4];
    o->live = (int64_t)std::llround(out[5]);
    o->gauss_res = out[6];
    o->wake_amp = out[7];
    o->nan_flag = nanf || !std::isfinite(out[0]) || !std::isfinite(out[1]);
    return BFPIC_OK;
  }

  static int axis_record(bfpic_ctx* h, int frame, double* out) {
    k_axis_record<R><<<(unsigned)cdiv(h->nz + 1, 256), 256, 0, h->stream>>>(
        h->g, fields(h), frame, h->gamma_b, h->beta_b, out);
    HIPCHK(h, hipGetLastError());
    return BFPIC_OK;
  }

  static int get_field(bfpic_ctx* h, int comp, double* out) {
    const Geo& g = h->g;
    const R* A;
    int half;
    if (comp < 6) {
      A = (const R*)h->F[comp];
      half = comp == 2 || comp == 3 || comp == 4;
    } else {
      A = (const R*)h->Jf[comp - 6];
      half = comp == 8;
    }
    k_get_field<R><<<(unsigned)cdiv((h->nz + 1) * g.plane, 256), 256, 0, h->stream>>>(g, A, out,
                                                                                     half);
    HIPCHK(h, hipGetLastError());
    return BFPIC_OK;
  }

  static int set_field(bfpic_ctx* h, int comp, const double* in) {
    const Geo& g = h->g;
    int half = comp == 2 || comp == 3 || comp == 4;
    k_set_field<R><<<(unsigned)cdiv((h->nz + 1) * g.plane, 256), 256, 0, h->stream>>>(
        g, (R*)h->F[comp], in, half);
    HIPCHK(h, hipGetLastError());
    return BFPIC_OK;
  }

  static int export_particles(bfpic_ctx* h, double* z, double* x, double* y, double* ux,
                              double* uy, double* uz, double* w, int* id) {
    if (h->slots_bound == 0) return BFPIC_OK;
    k_export<R, DIM><<<(unsigned)cdiv(h->slots_bound, 256), 256, 0, h->stream>>>(
        soa(h, h->cur), lattice(h), drift(h, h->step), h->u_b, h->counts, z, x, y, ux, uy, uz, w,
        id);
    HIPCHK(h, hipGetLastError());
    return BFPIC_OK;
  }
};

// Dispatch on (precision, dim, order).
#define BFPIC_DISPATCH(h, EXPR)                                                    \
  do {                                                                             \
    if ((h)->fp64) {                                                               \
      if ((h)->dim == 2) {                                                         \
        if ((h)->order == 1) { using I = Impl<double, 2, 1>; return EXPR; }        \
        else { using I = Impl<double, 2, 2>; return EXPR; }                        \
      } else {                                                                     \
        if ((h)->order == 1) { using I = Impl<double, 3, 1>; return EXPR; }        \
        else { using I = Impl<double, 3, 2>; return EXPR; }                        \
      }                                                                            \
    } else {                                                                       \
      if ((h)->dim == 2) {                                                         \
        if ((h)->order == 1) { using I = Impl<float, 2, 1>; return EXPR; }         \
        else { using I = Impl<float, 2, 2>; return EXPR; }                         \
      } else {                                                                     \
        if ((h)->order == 1) { using I = Impl<float, 3, 1>; return EXPR; }         \
        else { using I = Impl<float, 3, 2>; return EXPR; }                         \
      }                                                                            \
    }                                                                              \
  } while (0)

static int prepare_kernels(bfpic_ctx* h) { BFPIC_DISPATCH(h, I::prepare(h)); }
static int tape_bytes_of(bfpic_ctx* h, int nsteps, int interval, int64_t* out) {
  BFPIC_DISPATCH(h, (*out = I::tape_map(h, nullptr, nsteps, interval).total, BFPIC_OK));
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int bfpic_query_sizes(const bfpic_config* cfg, int64_t cap, bfpic_sizes* out) {
  std::string why;
  if (!out || cap < 1 || cap > 0x7fffffffLL || !check_cfg(cfg, why)) return BFPIC_ERR_ARG;
  bfpic_ctx tmp;
  derive(&tmp, cfg);
  plan(&tmp, cap, nullptr, out);
  return BFPIC_OK;
}

extern "C" int bfpic_create(const bfpic_config* cfg, int64_t cap, void* workspace,
                            int64_t workspace_bytes, void* stream, bfpic_ctx** out) {
  if (!out) return BFPIC_ERR_ARG;
  *out = nullptr;
  std::string why;
  if (cap < 1 || cap > 0x7fffffffLL || !check_cfg(cfg, why) || !workspace)
    return BFPIC_ERR_ARG;
  bfpic_ctx* h = new bfpic_ctx();
  derive(h, cfg);
  h->cap = cap;
  bfpic_sizes sz;
  plan(h, cap, nullptr, &sz);
  if (workspace_bytes < sz.workspace_bytes || ((uintptr_t)workspace & 255)) {
    delete h;
    return BFPIC_ERR_ARG;
  }
  h->ws = (uint8_t*)workspace;
  h->ws_bytes = workspace_bytes;
  plan(h, cap, h, nullptr);
  h->stream = (hipStream_t)stream;
  int dev = 0, lds = 65536;
  if (hipGetDevice(&dev) == hipSuccess) {
    h->device = dev;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
      h->lds_limit = (size_t)lds;
    // set-up of the static scratch on this device (retried by its first
    // use if it fails here)
    void* sp = nullptr;
    (void)static_scratch_of(dev, &sp);
  }
  if (h->lds_tiled > h->lds_limit && h->dim == 3) {
    // 3D tiles whose staged fields do not fit: gather from global memory and
    // keep only the FP64 (or int64) currents in LDS
    h->stage = false;
    h->lds_tiled = (size_t)3 * h->LZ * h->LX * std::max(h->LY, kGpd3LdsY) * 8;
  }
  if (h->lds_tiled > h->lds_limit) h->tiled = false;
  // the filter kernels may need more than 64 KB of LDS (3D, FP64, many passes)
  {
    int lim = (int)h->lds_limit;
    hipFuncSetAttribute((const void*)k_filter_grid<2, kF2Z, kF2X, 1>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void*)k_filter_grid<3, kF3, kF3, kF3>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)k_filter_grid_r3d<float, kF3>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)k_filter_grid_r3d<double, kF3>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    FiltK fk;
    fk.passes = cfg->filter_passes;
    fk.comp = cfg->filter_compensate;
    int H = fk.passes + (fk.comp && fk.passes > 0 ? 1 : 0);
    size_t need = h->dim == 2 ? 2 * 8 * (size_t)(kF2Z + 2 * H) * (kF2X + 2 * H)
                              : 2 * 8 * (size_t)(kF3 + 2 * H) * (kF3 + 2 * H) * (kF3 + 2 * H);
    if (need > h->lds_limit) {
      delete h;
      return BFPIC_ERR_UNSUPPORTED;
    }
  }
  prepare_kernels(h);

  *out = h;
  return BFPIC_OK;
}

extern "C" void bfpic_destroy(bfpic_ctx* h) {
  if (!h) return;
  for (int c = 0; c < kNumTimers; c++)
    for (auto& pr : h->ev[c]) {
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
  for (auto e : h->pool) hipEventDestroy(e);
  delete h;
}

extern "C" const char* bfpic_last_error(const bfpic_ctx* h) { return h ? h->err.c_str() : "null"; }

extern "C" int init_boosted_plasma(bfpic_ctx* h, double gamma_boost, const bfpic_density* n_e,
                                   const bfpic_laser* laser) {
  if (!h) return BFPIC_ERR_ARG;
  if (!(gamma_boost >= 1.0)) return fail(h, BFPIC_ERR_ARG, "gamma_boost must be >= 1");
  if (n_e && n_e->nknots == 1) return fail(h, BFPIC_ERR_ARG, "nknots must be 0 or >= 2");
  BFPIC_DISPATCH(h, I::init(h, gamma_boost, n_e, laser));
}

extern "C" int pic_step(bfpic_ctx* h, int32_t nsteps) {
  if (!h) return BFPIC_ERR_ARG;
  if (!h->inited) return fail(h, BFPIC_ERR_STATE, "pic_step before init_boosted_plasma");
  if (nsteps < 0) return fail(h, BFPIC_ERR_ARG, "nsteps < 0");
  BFPIC_DISPATCH(h, I::steps(h, nsteps));
}

extern "C" int moving_window_shift(bfpic_ctx* h, int32_t n) {
  if (!h) return BFPIC_ERR_ARG;
  if (!h->inited) return fail(h, BFPIC_ERR_STATE, "window shift before init");
  if (h->g.periodic_z && n != 0) return fail(h, BFPIC_ERR_ARG, "periodic z has no window");
  BFPIC_DISPATCH(h, I::shift(h, n));
}

extern "C" int bfpic_window_due(bfpic_ctx* h, int32_t* n) {
  if (!h || !n) return BFPIC_ERR_ARG;
  double t = (double)h->step * h->dt;
  *n = (int32_t)(std::floor((h->cfg.beta_window * t) / h->dz) - (double)h->window_cells);
  return BFPIC_OK;
}

extern "C" int diagnostics(bfpic_ctx* h, uint32_t mask, bfpic_diag* out, double* lineout) {
  (void)mask;
  if (!h || !out) return BFPIC_ERR_ARG;
  if (!h->inited) return fail(h, BFPIC_ERR_STATE, "diagnostics before init");
  BFPIC_DISPATCH(h, I::diag(h, out, lineout));
}

extern "C" int diagnostics_noalloc(bfpic_ctx* h, uint32_t mask, bfpic_diag* out,
                                   double* lineout) {
  (void)mask;
  if (!h || !out) return BFPIC_ERR_ARG;
  if (!h->inited) return fail(h, BFPIC_ERR_STATE, "diagnostics before init");
  int cur = -1;
  HIPCHK(h, hipGetDevice(&cur));
  if (cur != h->device) return fail(h, BFPIC_ERR_STATE, "the context's device is not current");
  void* base = nullptr;
  hipError_t e = static_scratch_of(cur, &base);
  if (e != hipSuccess)
    return fail(h, BFPIC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e));
  BFPIC_DISPATCH(h, I::diag_static(h, out, lineout, (uint8_t*)base));
}

extern "C" int bfpic_axis_record(bfpic_ctx* h, int32_t frame, double* out, bfpic_axis_meta* meta) {
  if (!h || !out || (frame != 0 && frame != 1)) return BFPIC_ERR_ARG;
  if (!h->inited) return fail(h, BFPIC_ERR_STATE, "axis record before init");
  if (meta) {
    meta->step = h->step;
    meta->t_prime = (double)h->step * h->dt;
    meta->z0_prime = (double)h->window_cells * h->dz;
    meta->dz_prime = h->dz;
    meta->n = h->nz + 1;
    meta->gamma_b = h->gamma_b;
    meta->beta_b = h->beta_b;
  }
  BFPIC_DISPATCH(h, I::axis_record(h, frame, out));
}

extern "C" int bfpic_witness_bind(bfpic_ctx* h, int32_t n, double* state_dev) {
  if (!h || n < 0 || (n > 0 && !state_dev)) return BFPIC_ERR_ARG;
  if (!h->inited) return fail(h, BFPIC_ERR_STATE, "witness bind before init");
  h->wit = n > 0 ? state_dev : nullptr;
  h->nwit = n;
  return BFPIC_OK;
}

extern "C" int bfpic_witness_lab(bfpic_ctx* h, double* out_dev) {
  if (!h || !out_dev) return BFPIC_ERR_ARG;
  if (h->nwit == 0) return fail(h, BFPIC_ERR_STATE, "no witnesses bound");
  k_witness_lab<<<(unsigned)cdiv(h->nwit, 256), 256, 0, h->stream>>>(
      h->wit, h->nwit, (double)h->step * h->dt, (double)h->window_cells * h->dz, h->dz,
      h->gamma_b, h->beta_b, out_dev);
  if (hipGetLastError() != hipSuccess) return fail(h, BFPIC_ERR_HIP, "witness lab launch");
  return BFPIC_OK;
}

extern "C" int bfpic_back_transform(bfpic_ctx* h, const double* rec, const double* tp,
                                    const double* z0, int64_t nrec, int32_t n, double dz,
                                    double gamma_b, double t0, double dt, int32_t nt,
                                    double zeta0, double dzeta, int32_t nzeta, double v_window,
                                    double* out) {
  if (!h) return BFPIC_ERR_ARG;
  if (!rec || !tp || !z0 || !out || nrec < 2 || n < 2 || nt < 1 || nzeta < 1 || !(dz > 0.0) ||
      !(gamma_b >= 1.0))
    return fail(h, BFPIC_ERR_ARG, "back transform arguments");
  BackK K;
  K.rec = rec;
  K.tp = tp;
  K.z0 = z0;
  K.nrec = nrec;
  K.n = n;
  K.dz = dz;
  K.gamma = gamma_b;
  K.beta = bfpic_beta(gamma_b);
  K.t0 = t0;
  K.dt = dt;
  K.zeta0 = zeta0;
  K.dzeta = dzeta;
  K.vw = v_window;
  K.nt = nt;
  K.nzeta = nzeta;
  const int64_t tot = (int64_t)nt * nzeta;
  k_back_transform<<<(unsigned)cdiv(tot, 256), 256, 0, h->stream>>>(K, out);
  HIPCHK(h, hipGetLastError());
  return BFPIC_OK;
}

extern "C" int bfpic_axis_spectrum(bfpic_ctx* h, const double* rec, int64_t nrec, int32_t n,
                                   int32_t m, double* out) {
  if (!h) return BFPIC_ERR_ARG;
  if (!rec || !out || nrec < 1 || m < 2 || m > 8192 || (m & (m - 1)) != 0 || n < 1 || n > m ||
      nrec > 0x7fffffff)
    return fail(h, BFPIC_ERR_ARG, "spectrum arguments");
  int logm = 0;
  while ((1 << logm) < m) logm++;
  const size_t lds = (size_t)2 * m * sizeof(double);
  HIPCHK(h, hipFuncSetAttribute((const void*)k_axis_spectrum,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  k_axis_spectrum<<<(unsigned)nrec, 256, lds, h->stream>>>(rec, n, m, logm, out);
  HIPCHK(h, hipGetLastError());
  return BFPIC_OK;
}

extern "C" int bfpic_get_field(bfpic_ctx* h, int32_t comp, double* out) {
  if (!h || !out || comp < 0 || comp > 8) return BFPIC_ERR_ARG;
  BFPIC_DISPATCH(h, I::get_field(h, comp, out));
}

extern "C" int bfpic_set_field(bfpic_ctx* h, int32_t comp, const double* in) {
  if (!h || !in || comp < 0 || comp > 5) return BFPIC_ERR_ARG;
  BFPIC_DISPATCH(h, I::set_field(h, comp, in));
}

extern "C" int bfpic_num_slots(bfpic_ctx* h, int64_t* n) {
  if (!h || !n) return BFPIC_ERR_ARG;
  int c = 0;
  HIPCHK(h, hipMemcpyAsync(&c, h->counts, 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  *n = c;
  return BFPIC_OK;
}

extern "C" int bfpic_get_particles(bfpic_ctx* h, double* z, double* x, double* y, double* ux,
                                   double* uy, double* uz, double* w, int32_t* id) {
  if (!h || !z || !x || !y || !ux || !uy || !uz || !w || !id) return BFPIC_ERR_ARG;
  BFPIC_DISPATCH(h, I::export_particles(h, z, x, y, ux, uy, uz, w, id));
}

extern "C" int bfpic_sort(bfpic_ctx* h) {
  if (!h) return BFPIC_ERR_ARG;
  if (!h->inited) return fail(h, BFPIC_ERR_STATE, "sort before init");
  BFPIC_DISPATCH(h, I::sort(h));
}

// ---------------------------------------------------------------------------
// Checkpoint / resume.  A state blob is one caller-owned device buffer: a
// header (identity of the configuration, the host schedule, the boost and
// density parameters, the fixed-point scale), then E and B with their guard
// rows, the live particle slots and the device counters.  Currents, the
// overflow grid and the Mur and shift buffers are rebuilt within each step
// and are not state; neither are bound witnesses (the caller's).
// ---------------------------------------------------------------------------
namespace {
constexpr uint64_t kStateMagic = 0x3153544349504642ull;  // "BFPICTS1"
constexpr int64_t kStateHead = 4096;

struct StateHeader {
  uint64_t magic;
  int64_t total;
  bfpic_config cfg;
  int64_t cap, slots;
  int64_t step, window_cells, next_col, slots_bound, tail_bound;
  double gamma_b, beta_b, u_b, sb, laser_a0, fx_scale, fx_inv;
  int32_t has_plasma, ndisp;
  DensityK dens;
};
static_assert(sizeof(StateHeader) <= kStateHead, "state header");

struct StateMap {
  int64_t field, id, comp, counts, total;
};

StateMap state_map(const bfpic_ctx* h, int64_t slots) {
  const int64_t es = h->fp64 ? 8 : 4;
  StateMap m;
  m.field = align256(h->g.rows * h->g.plane * es);
  m.id = align256(std::max<int64_t>(slots, 1) * 4);
  m.comp = align256(std::max<int64_t>(slots, 1) * es);
  const int ndisp = h->dim == 3 ? 3 : 2;
  m.counts = 256;
  m.total = kStateHead + 6 * m.field + m.id + (int64_t)(ndisp + 4) * m.comp + m.counts;
  return m;
}

bool same_physics(const bfpic_config& a, const bfpic_config& b) {
  return a.dim == b.dim && a.nz == b.nz && a.nx == b.nx && a.ny == b.ny && a.dz == b.dz &&
         a.dx == b.dx && a.dy == b.dy && a.cfl == b.cfl && a.shape_order == b.shape_order &&
         a.filter_passes == b.filter_passes && a.filter_compensate == b.filter_compensate &&
         a.precision == b.precision && a.deterministic == b.deterministic &&
         a.z_boundary == b.z_boundary && a.ppc == b.ppc && a.load == b.load &&
         a.seed == b.seed && a.beta_window == b.beta_window && a.auto_window == b.auto_window &&
         a.gather_form == b.gather_form;
}

// Device arrays of the state in blob order: E, B, id, displacements,
// momenta, weight.
int state_arrays(bfpic_ctx* h, int64_t slots, void* ptr[16], int64_t bytes[16]) {
  const int64_t es = h->fp64 ? 8 : 4;
  int n = 0;
  for (int c = 0; c < 6; c++) {
    ptr[n] = h->F[c];
    bytes[n++] = h->g.rows * h->g.plane * es;
  }
  ptr[n] = h->pid[h->cur];
  bytes[n++] = slots * 4;
  const int ndisp = h->dim == 3 ? 3 : 2;
  for (int a = 0; a < ndisp; a++) {
    ptr[n] = h->pxi[h->cur][a];
    bytes[n++] = slots * es;
  }
  for (int a = 0; a < 3; a++) {
    ptr[n] = h->pdu[h->cur][a];
    bytes[n++] = slots * es;
  }
  ptr[n] = h->pw[h->cur];
  bytes[n++] = slots * es;
  return n;
}
}  // namespace

static int reset_device_of(bfpic_ctx* h) { BFPIC_DISPATCH(h, I::reset_device(h)); }

extern "C" int bfpic_state_bytes(bfpic_ctx* h, int64_t* bytes) {
  if (!h || !bytes) return BFPIC_ERR_ARG;
  if (!h->inited) return fail(h, BFPIC_ERR_STATE, "state size before init");
  *bytes = state_map(h, h->slots_bound).total;
  return BFPIC_OK;
}

extern "C" int pic_save(bfpic_ctx* h, void* blob_dev, int64_t blob_bytes) {
  if (!h || !blob_dev) return BFPIC_ERR_ARG;
  if (!h->inited) return fail(h, BFPIC_ERR_STATE, "save before init");
  const StateMap m = state_map(h, h->slots_bound);
  if (blob_bytes < m.total || ((uintptr_t)blob_dev & 255))
    return fail(h, BFPIC_ERR_ARG, "state blob too small or misaligned");
  StateHeader hd{};
  hd.magic = kStateMagic;
  hd.total = m.total;
  hd.cfg = h->cfg;
  hd.cap = h->cap;
  hd.slots = h->slots_bound;
  hd.step = h->step;
  hd.window_cells = h->window_cells;
  hd.next_col = h->next_col;
  hd.slots_bound = h->slots_bound;
  hd.tail_bound = h->tail_bound;
  hd.gamma_b = h->gamma_b;
  hd.beta_b = h->beta_b;
  hd.u_b = h->u_b;
  hd.sb = h->sb;
  hd.laser_a0 = h->laser_a0;
  hd.fx_scale = h->fx_scale;
  hd.fx_inv = h->fx_inv;
  hd.has_plasma = h->has_plasma ? 1 : 0;
  hd.ndisp = h->dim == 3 ? 3 : 2;
  hd.dens = h->dens;
  uint8_t* b = (uint8_t*)blob_dev;
  HIPCHK(h, hipMemcpyAsync(b, &hd, sizeof(hd), hipMemcpyHostToDevice, h->stream));
  void* ptr[16];
  int64_t bytes[16];
  const int n = state_arrays(h, h->slots_bound, ptr, bytes);
  int64_t o = kStateHead;
  for (int q = 0; q < n; q++) {
    if (bytes[q] > 0)
      HIPCHK(h, hipMemcpyAsync(b + o, ptr[q], (size_t)bytes[q], hipMemcpyDeviceToDevice, h->stream));
    o += q < 6 ? m.field : (q == 6 ? m.id : m.comp);
  }
  HIPCHK(h, hipMemcpyAsync(b + o, h->counts, 16 * 4, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));  // the header's host copy
  return BFPIC_OK;
}

extern "C" int pic_load(bfpic_ctx* h, const void* blob_dev, int64_t blob_bytes) {
  if (!h || !blob_dev) return BFPIC_ERR_ARG;
  if (blob_bytes < kStateHead || ((uintptr_t)blob_dev & 255))
    return fail(h, BFPIC_ERR_ARG, "state blob too small or misaligned");
  StateHeader hd{};
  HIPCHK(h, hipMemcpyAsync(&hd, blob_dev, sizeof(hd), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (hd.magic != kStateMagic) return fail(h, BFPIC_ERR_ARG, "not a state blob");
  if (!same_physics(hd.cfg, h->cfg))
    return fail(h, BFPIC_ERR_ARG, "state blob of another configuration");
  if (hd.slots < 0 || hd.slots > h->cap)
    return fail(h, BFPIC_ERR_CAPACITY, "state blob holds more slots than the capacity");
  const StateMap m = state_map(h, hd.slots);
  if (hd.total != m.total || blob_bytes < m.total)
    return fail(h, BFPIC_ERR_ARG, "state blob size does not match its header");
  h->step = hd.step;
  h->window_cells = hd.window_cells;
  h->next_col = hd.next_col;
  h->slots_bound = hd.slots_bound;
  h->tail_bound = hd.tail_bound;
  h->gamma_b = hd.gamma_b;
  h->beta_b = hd.beta_b;
  h->u_b = hd.u_b;
  h->sb = hd.sb;
  h->laser_a0 = hd.laser_a0;
  h->fx_scale = hd.fx_scale;
  h->fx_inv = hd.fx_inv;
  h->has_plasma = hd.has_plasma != 0;
  h->dens = hd.dens;
  h->adj_ready = false;
  h->no_sort = false;
  h->have_sort = false;
  const int rz = reset_device_of(h);
  if (rz) return rz;
  const uint8_t* b = (const uint8_t*)blob_dev;
  void* ptr[16];
  int64_t bytes[16];
  const int n = state_arrays(h, hd.slots, ptr, bytes);
  int64_t o = kStateHead;
  for (int q = 0; q < n; q++) {
    if (bytes[q] > 0)
      HIPCHK(h, hipMemcpyAsync(ptr[q], b + o, (size_t)bytes[q], hipMemcpyDeviceToDevice, h->stream));
    o += q < 6 ? m.field : (q == 6 ? m.id : m.comp);
  }
  HIPCHK(h, hipMemcpyAsync(h->counts, b + o, 16 * 4, hipMemcpyDeviceToDevice, h->stream));
  h->inited = true;
  // the tile structures follow the particle order: rebuild them
  return bfpic_sort(h);
}

extern "C" int bfpic_last_sort(bfpic_ctx* h, int32_t* key_dev, int32_t* id_dev, int32_t* perm_dev,
                               int64_t* n, int64_t* n_live, int64_t* tz_min, int32_t* ntz) {
  if (!h || !key_dev || !id_dev || !perm_dev || !n || !n_live || !tz_min || !ntz)
    return BFPIC_ERR_ARG;
  if (!h->have_sort) return fail(h, BFPIC_ERR_STATE, "no sort yet");
  int c[3];
  HIPCHK(h, hipMemcpyAsync(c, h->counts, sizeof(c), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int nsrc = c[2];
  HIPCHK(h, hipMemcpyAsync(key_dev, h->key, (size_t)nsrc * 4, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(id_dev, h->pid[1 - h->cur], (size_t)nsrc * 4, hipMemcpyDeviceToDevice,
                           h->stream));
  int nl = 0;
  HIPCHK(h, hipMemcpyAsync(&nl, h->off + h->last_sort_nkeys, 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, hipMemcpyAsync(perm_dev, h->final_perm, (size_t)nl * 4, hipMemcpyDeviceToDevice,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  *n = nsrc;
  *n_live = nl;
  *tz_min = h->last_sort_tzmin;
  *ntz = h->last_sort_ntz;
  return BFPIC_OK;
}

extern "C" int bfpic_sort_permutation(bfpic_ctx* h, int32_t* perm_dev, int64_t* n_live) {
  if (!h || !perm_dev || !n_live) return BFPIC_ERR_ARG;
  if (!h->have_sort) return fail(h, BFPIC_ERR_STATE, "no sort yet");
  int nl = 0;
  HIPCHK(h, hipMemcpyAsync(&nl, h->off + h->last_sort_nkeys, 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, hipMemcpyAsync(perm_dev, h->final_perm, (size_t)nl * 4, hipMemcpyDeviceToDevice,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  *n_live = nl;
  return BFPIC_OK;
}

extern "C" int bfpic_tile_shape(const bfpic_ctx* h, int32_t* tz, int32_t* tx, int32_t* ty) {
  if (!h || !tz || !tx || !ty) return BFPIC_ERR_ARG;
  *tz = h->TZ;
  *tx = h->TX;
  *ty = h->TY;
  return BFPIC_OK;
}

extern "C" int bfpic_kernel_timing(bfpic_ctx* h, int32_t enable) {
  if (!h) return BFPIC_ERR_ARG;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int c = 0; c < kNumTimers; c++) {
    for (auto& pr : h->ev[c]) {
      h->pool.push_back(pr.first);
      h->pool.push_back(pr.second);
    }
    h->ev[c].clear();
  }
  h->timing = enable != 0;
  return BFPIC_OK;
}

extern "C" int bfpic_kernel_time(bfpic_ctx* h, int32_t cls, double* total_ms, int64_t* launches) {
  if (!h || cls < 0 || cls >= kNumTimers || !total_ms || !launches) return BFPIC_ERR_ARG;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  double tot = 0.0;
  for (auto& pr : h->ev[cls]) {
    float ms = 0.f;
    HIPCHK(h, hipEventElapsedTime(&ms, pr.first, pr.second));
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)h->ev[cls].size();
  return BFPIC_OK;
}

// ---------------------------------------------------------------------------
// Adjoint
// ---------------------------------------------------------------------------
extern "C" int bfpic_adjoint_tape_bytes(bfpic_ctx* h, int32_t nsteps, int32_t interval,
                                        int64_t* bytes) {
  if (!h || !bytes || nsteps < 1 || interval < 1) return BFPIC_ERR_ARG;
  return tape_bytes_of(h, nsteps, interval, bytes);
}

extern "C" int bfpic_forward_loss(bfpic_ctx* h, int32_t nsteps, int32_t interval,
                                  const bfpic_loss* loss, void* tape, int64_t tape_bytes,
                                  double* loss_out) {
  if (!h || !loss || !loss_out) return BFPIC_ERR_ARG;
  BFPIC_DISPATCH(h, I::forward_loss(h, nsteps, interval, loss, tape, tape_bytes, loss_out));
}

extern "C" int bfpic_antenna(bfpic_ctx* h, const bfpic_laser* laser, int32_t row) {
  if (!h) return BFPIC_ERR_ARG;
  BFPIC_DISPATCH(h, I::set_antenna(h, laser, row));
}

extern "C" int bfpic_adjoint_per_direction(bfpic_ctx* h, int32_t enable) {
  if (!h) return BFPIC_ERR_ARG;
  h->adj_per_direction = enable != 0;
  return BFPIC_OK;
}

extern "C" int pic_step_adjoint(bfpic_ctx* h, double* dL_da0, double* dL_dn, int32_t nn) {
  if (!h || !dL_da0 || !dL_dn) return BFPIC_ERR_ARG;
  BFPIC_DISPATCH(h, I::adjoint(h, dL_da0, dL_dn, nn));
}
