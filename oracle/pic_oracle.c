/*
 * pic_oracle.c -- plain FP64 CPU particle-in-cell oracle (test infrastructure).
 *
 * Only the test suite, the smoke check and the CPU baseline leg of the
 * benchmark use this file.  It shares no code with the HIP library.
 *
 * Every function below states the passage or textbook method it follows.
 * The paper defers its numerical scheme to companion papers (end of the
 * introduction; first paragraph of "Mitigation of a numerical instability"),
 * so the step is the standard explicit electromagnetic PIC cycle the method
 * runs in the boosted frame: gather -> Boris push -> move -> Esirkepov
 * deposit -> binomial current filter -> Yee update.  Where the paper leaves
 * a choice open, the function that makes it states the reading it takes.
 *
 * Conventions
 *   positions: absolute, in cells, relative to the current grid origin, held
 *   in x87 extended precision (long double, 64-bit significand): at 8192
 *   cells an FP64 coordinate resolves 1.8e-12 cell, about 1e-4 of the
 *   distance a boosted pair's electron moves away from its partner in one
 *   step at gamma_b = 130, while the extended one resolves 9e-16 cell.  Every
 *   shape factor is evaluated in FP64 on the offset from its stencil base,
 *   formed in extended precision.
 *   grid node (i, j, k) of a component sits at ((i+sz)dz, (j+sx)dx, (k+sy)dy)
 *   with the Yee offsets of the table SIG below; y is absent in 2D.
 *   Fields are stored for rows i = -G .. nz+G; rows outside the physical
 *   domain stay zero when the z boundary is not periodic.
 */
#include "pic_oracle.h"

#include <complex.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define G_ROWS 6

/* Yee staggering (z, x, y) of every component, in cells. */
static const double SIG[ORC_NCOMP][3] = {
    {0.0, 0.5, 0.0}, /* Ex */
    {0.0, 0.0, 0.5}, /* Ey */
    {0.5, 0.0, 0.0}, /* Ez */
    {0.5, 0.0, 0.5}, /* Bx */
    {0.5, 0.5, 0.0}, /* By */
    {0.0, 0.5, 0.5}, /* Bz */
    {0.0, 0.5, 0.0}, /* Jx */
    {0.0, 0.0, 0.5}, /* Jy */
    {0.5, 0.0, 0.0}, /* Jz */
};

typedef long double xpos; /* particle coordinates (see the conventions above) */

/* floor of an extended-precision coordinate as an integer: truncation toward
 * zero, one lower for a negative non-integer (|x| < 2^62) */
static int64_t ifloorx(xpos x) {
  int64_t i = (int64_t)x;
  return x < (xpos)i ? i - 1 : i;
}

struct orc_sim {
  orc_config c;
  int nyy;        /* ny in 3D, 1 in 2D */
  int nzs;        /* stored rows */
  int64_t plane;  /* nx * nyy */
  double* F[ORC_NCOMP];
  double* rho;    /* diagnostics scratch, same shape as one component */
  /* particle pairs: electron (e) and its ion partner (i) */
  int64_t np, cap;
  xpos *ze, *xe, *ye, *zi, *xi, *yi;
  double *uz, *ux, *uy, *w;
  int64_t* id;
  int64_t step;
  double window_cells;
  int64_t next_col;
  int has_plasma;
  /* density profile copy */
  double n_uniform;
  int nknots;
  double* kz;
  double* kn;
  double du0[3];
  double ch_depth, ch_radius;
  /* per-thread current buffers of the parallel particle loop (thread t > 0
   * deposits into tJ[t-1][comp]; thread 0 into the grid's own J) */
  int nthreads;
  double** tJ;
  /* laser antenna: a current sheet on grid row ant_row (< 0: none) */
  int ant_row;
  orc_laser ant;
};

/* ------------------------------------------------------------------------ */
/* Boost helper.  Lorentz boost along +z (introduction; section "Effect of   */
/* the hyperbolic rotation": the frame change is a hyperbolic rotation).      */
/* ------------------------------------------------------------------------ */

double orc_beta_of_gamma(double gamma) { return sqrt(gamma * gamma - 1.0) / gamma; }

/* 1 - beta = 1 / (gamma^2 (1 + beta)), free of cancellation at large gamma. */
double orc_one_minus_beta(double gamma) {
  double beta = orc_beta_of_gamma(gamma);
  return 1.0 / (gamma * gamma * (1.0 + beta));
}

/* A plasma at rest in the lab drifts at -beta_b in the boosted frame. */
double orc_drift_u(double gamma_b) { return -sqrt(gamma_b * gamma_b - 1.0); }

/* Laser group velocity in a cold plasma (1D): gamma_g = omega0/omega_p = 1/sqrt(n)
 * in normalised units; the paper's gamma_g ~ 13.2 at 1e19 cm^-3 follows. */
double orc_group_gamma(double n_lab) { return 1.0 / sqrt(n_lab); }

/* Boosted-frame group velocity beta'_g = (beta_g - beta_b) / (1 - beta_g beta_b),
 * with both differences written without cancellation:
 *   beta_g - beta_b = (1/gamma_b^2 - 1/gamma_g^2) / (beta_g + beta_b)
 *   1 - beta_g beta_b = (1/gamma_g^2 + 1/gamma_b^2 + (beta_g - beta_b)^2) / 2   */
double orc_boosted_group_beta(double gamma_b, double n_lab) {
  double gg = orc_group_gamma(n_lab);
  double bg = orc_beta_of_gamma(gg), bb = orc_beta_of_gamma(gamma_b);
  double ig2 = 1.0 / (gg * gg), ib2 = 1.0 / (gamma_b * gamma_b);
  double num = (ib2 - ig2) / (bg + bb);
  double den = 0.5 * (ig2 + ib2 + num * num);
  return num / den;
}

/* Longitudinal resolution set against the vacuum laser wavelength (section
 * "Mitigation of a numerical instability"): the boosted wavelength is
 * gamma_b (1 + beta_b) lambda0, resolved by cells_per_wavelength cells. */
double orc_boosted_dz(double gamma_b, double lambda0, double cells_per_wavelength) {
  double beta = orc_beta_of_gamma(gamma_b);
  return gamma_b * (1.0 + beta) * lambda0 / cells_per_wavelength;
}

/* Yee Courant limit dt_max = 1/sqrt(sum 1/d^2); dt = cfl * dt_max. */
double orc_yee_dt(int32_t dim, double dz, double dx, double dy, double cfl) {
  double s = 1.0 / (dz * dz) + 1.0 / (dx * dx);
  if (dim == 3) s += 1.0 / (dy * dy);
  return cfl / sqrt(s);
}

/* Linear-theory depletion length L_d = lambda_p^3 / (2 lambda0^2) (introduction),
 * lambda_p = 2 pi / sqrt(n), lambda0 = 2 pi in units of c/omega0. */
double orc_depletion_length(double n_lab) {
  double lp = 2.0 * M_PI / sqrt(n_lab), l0 = 2.0 * M_PI;
  return lp * lp * lp / (2.0 * l0 * l0);
}

/* ------------------------------------------------------------------------ */
/* Counter-based generator: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).    */
/* State after n increments is seed + n * 0x9E3779B97F4A7C15; the output is  */
/* the published 64-bit finaliser of that state.                              */
/* ------------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t seed, uint64_t n) {
  uint64_t z = seed + n * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* In-cell offset of slot s of lattice cell (k, l, j) along axis (0 z, 1 x,
 * 2 y): a 24-bit field of a generator output, times 2^-24, so that the value
 * is exact in FP32 and FP64.  With id the slot's running index, output
 * 2 id + 1 gives z (bits 63..40) and x (bits 39..16), output 2 id + 2 gives
 * y (bits 63..40). */
double orc_cell_offset(uint64_t seed, int64_t k, int64_t l, int64_t j, int32_t s,
                       int32_t axis, int32_t nx, int32_t nyy, int32_t ppc) {
  uint64_t id = (((uint64_t)k * (uint64_t)nyy + (uint64_t)l) * (uint64_t)nx +
                 (uint64_t)j) * (uint64_t)ppc + (uint64_t)s;
  uint64_t r = orc_splitmix64(seed, 2ULL * id + 1ULL + (axis == 2 ? 1ULL : 0ULL));
  uint64_t field = axis == 1 ? (r >> 16) & 0xFFFFFFULL : r >> 40;
  return (double)field * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------------ */
/* Shape functions: the B-splines of order 0 (nearest grid point: 1 on        */
/* [-1/2, 1/2), the half-open cell of the node), 1 (linear, max(0, 1-|d|))    */
/* and 2 (quadratic).                                                          */
/* ------------------------------------------------------------------------ */
double orc_shape(int32_t order, double d) {
  double a = fabs(d);
  if (order == 0) return (d >= -0.5 && d < 0.5) ? 1.0 : 0.0;
  if (order == 1) return a < 1.0 ? 1.0 - a : 0.0;
  if (a <= 0.5) return 0.75 - a * a;
  if (a < 1.5) {
    double b = 1.5 - a;
    return 0.5 * b * b;
  }
  return 0.0;
}

/* ------------------------------------------------------------------------ */
/* Relativistic Boris push (Boris 1970), vectors ordered (x, y, z), m = 1:   */
/*   u- = u + h E, h = q dt / 2;  t = h B / gamma(u-);  s = 2 t / (1 + t^2)   */
/*   u' = u- + u- x t;  u+ = u- + u' x s;  u_new = u+ + h E                  */
/* ------------------------------------------------------------------------ */
static void cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

void orc_boris(double q, double dt, const double E[3], const double B[3], double u[3]) {
  double h = 0.5 * q * dt;
  double um[3], t[3], s[3], c1[3], up[3], c2[3];
  for (int a = 0; a < 3; a++) um[a] = u[a] + h * E[a];
  double g = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  for (int a = 0; a < 3; a++) t[a] = h * B[a] / g;
  double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  for (int a = 0; a < 3; a++) s[a] = 2.0 * t[a] / (1.0 + t2);
  cross(um, t, c1);
  for (int a = 0; a < 3; a++) up[a] = um[a] + c1[a];
  cross(up, s, c2);
  for (int a = 0; a < 3; a++) u[a] = um[a] + c2[a] + h * E[a];
}

/* ------------------------------------------------------------------------ */
/* Stable sort by (key, id): a comparison sort with the source index as the  */
/* final tie-break, so the order is unique.                                   */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t key, id; int32_t idx; } sort_rec;

static int cmp_rec(const void* pa, const void* pb) {
  const sort_rec* a = (const sort_rec*)pa;
  const sort_rec* b = (const sort_rec*)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  if (a->id != b->id) return a->id < b->id ? -1 : 1;
  return a->idx < b->idx ? -1 : (a->idx > b->idx);
}

void orc_sort_perm(int64_t n, const int32_t* key, const int32_t* id, int32_t* perm) {
  sort_rec* r = (sort_rec*)malloc((size_t)(n > 0 ? n : 1) * sizeof(sort_rec));
  for (int64_t p = 0; p < n; p++) {
    r[p].key = key[p];
    r[p].id = id[p];
    r[p].idx = (int32_t)p;
  }
  qsort(r, (size_t)n, sizeof(sort_rec), cmp_rec);
  for (int64_t p = 0; p < n; p++) perm[p] = r[p].idx;
  free(r);
}

/* ------------------------------------------------------------------------ */
/* Grid access                                                                */
/* ------------------------------------------------------------------------ */
static int64_t wrapi(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

/* Storage index of node (i, j, k) or -1 if the row is outside storage. */
static int64_t node(const orc_sim* s, int64_t i, int64_t j, int64_t k) {
  const orc_config* c = &s->c;
  if (c->zbc == 0) i = wrapi(i, c->nz);
  else if (i < -G_ROWS || i > c->nz + G_ROWS) return -1;
  j = wrapi(j, c->nx);
  k = (c->dim == 3) ? wrapi(k, c->ny) : 0;
  return ((i + G_ROWS) * c->nx + j) * s->nyy + k;
}

static double fget(const orc_sim* s, int comp, int64_t i, int64_t j, int64_t k) {
  int64_t n = node(s, i, j, k);
  return n < 0 ? 0.0 : s->F[comp][n];
}

static void add_at(const orc_sim* s, double* A, int64_t i, int64_t j, int64_t k, double v) {
  int64_t n = node(s, i, j, k);
  if (n >= 0) A[n] += v;
}

/* Physical domain rows of a component with z offset sz: [0, nz] for integer
 * z (both boundary planes carry the tangential E), [0, nz-1] for half-integer
 * z; [0, nz-1] for every component when z is periodic. */
static int row_lo(const orc_sim* s, double sz) { (void)s; (void)sz; return 0; }
static int row_hi(const orc_sim* s, double sz) {
  if (s->c.zbc == 0) return s->c.nz - 1;
  return sz == 0.0 ? s->c.nz : s->c.nz - 1;
}
static int in_domain(const orc_sim* s, double sz, int64_t i) {
  return i >= row_lo(s, sz) && i <= row_hi(s, sz);
}

/* ------------------------------------------------------------------------ */
/* Gather: F_p = sum_nodes F(node) S(z - i - sz) S(x - j - sx) [S(y - k - sy)]*/
/* Momentum-conserving form: every axis with the deposit's shape order.      */
/* Energy-conserving (Galerkin) form: an axis on which the component sits at */
/* half-integer nodes (s = 1/2) takes the shape of one order lower, the      */
/* shape that the charge-conserving current of that component has along it   */
/* (Esirkepov's J_z is a z-difference of the charge shape, so along z it      */
/* carries the integral of S^l, a shape of order l - 1 on the half nodes).    */
/* ------------------------------------------------------------------------ */
static int axis_order(const orc_sim* s, int comp, int axis) {
  int o = s->c.order;
  return (s->c.gather == 1 && SIG[comp][axis] == 0.5) ? o - 1 : o;
}

static double gather(const orc_sim* s, int comp, xpos z, xpos x, xpos y) {
  const orc_config* c = &s->c;
  const int oz = axis_order(s, comp, 0), ox = axis_order(s, comp, 1), oy = axis_order(s, comp, 2);
  xpos pz = z - SIG[comp][0], px = x - SIG[comp][1], py = y - SIG[comp][2];
  int64_t i0 = ifloorx(pz) - 2, j0 = ifloorx(px) - 2;
  int64_t k0 = ifloorx(py) - 2;
  /* offsets from the stencil base, small enough for FP64 */
  double lz = (double)(pz - (xpos)i0), lx = (double)(px - (xpos)j0), ly = (double)(py - (xpos)k0);
  double sum = 0.0;
  for (int a = 0; a < 6; a++) {
    double wz = orc_shape(oz, lz - (double)a);
    if (wz == 0.0) continue;
    for (int b = 0; b < 6; b++) {
      double wx = orc_shape(ox, lx - (double)b);
      if (wx == 0.0) continue;
      if (c->dim == 2) {
        sum += fget(s, comp, i0 + a, j0 + b, 0) * wz * wx;
      } else {
        for (int d = 0; d < 6; d++) {
          double wy = orc_shape(oy, ly - (double)d);
          if (wy == 0.0) continue;
          sum += fget(s, comp, i0 + a, j0 + b, k0 + d) * wz * wx * wy;
        }
      }
    }
  }
  return sum;
}

/* ------------------------------------------------------------------------ */
/* Esirkepov charge-conserving deposit (Esirkepov, CPC 135, 144, 2001).       */
/* On the charge lattice (integer nodes) with S0 / S1 the old / new shape     */
/* factors and dS = S1 - S0:                                                  */
/*  2D: Wz = dSz (S0x + dSx/2), Wx = dSx (S0z + dSz/2),                        */
/*      Wy = S0z S0x + dSz S0x/2 + S0z dSx/2 + dSz dSx/3                       */
/*      Jz(i+1/2) = Jz(i-1/2) - q w Wz / (dx dt);  Jx likewise with dz;       */
/*      Jy(i, j) += q w vy Wy / (dz dx)                                       */
/*  3D: Wz = dSz (S0x S0y + dSx S0y/2 + S0x dSy/2 + dSx dSy/3), cyclic;       */
/*      prefix sums scaled by q w / (d_other1 d_other2 dt).                   */
/* ------------------------------------------------------------------------ */
#define STN 12

static void shape_row(int order, xpos p0, xpos p1, int64_t* lo, int* n, double* S0,
                      double* S1) {
  int64_t a = ifloorx(p0 < p1 ? p0 : p1) - 2;
  int64_t b = ifloorx(p0 > p1 ? p0 : p1) + 3;
  *lo = a;
  *n = (int)(b - a + 1);
  if (*n > STN) *n = STN; /* displacements are below one cell per step */
  double l0 = (double)(p0 - (xpos)a), l1 = (double)(p1 - (xpos)a);
  for (int m = 0; m < *n; m++) {
    S0[m] = orc_shape(order, l0 - (double)m);
    S1[m] = orc_shape(order, l1 - (double)m);
  }
}

static void deposit_2d(const orc_sim* s, double* const* J, double q, double w, double vy,
                       xpos z0, xpos x0, xpos z1, xpos x1) {
  const orc_config* c = &s->c;
  int64_t lz, lx;
  int nz_, nx_;
  double S0z[STN], S1z[STN], S0x[STN], S1x[STN];
  shape_row(c->order, z0, z1, &lz, &nz_, S0z, S1z);
  shape_row(c->order, x0, x1, &lx, &nx_, S0x, S1x);
  double cz = -q * w / (c->dx * c->dt);
  double cx = -q * w / (c->dz * c->dt);
  double cy = q * w * vy / (c->dz * c->dx);
  /* Jz: prefix along z for every x node */
  for (int b = 0; b < nx_; b++) {
    double dSx = S1x[b] - S0x[b], acc = 0.0;
    for (int a = 0; a < nz_; a++) {
      double dSz = S1z[a] - S0z[a];
      acc += cz * dSz * (S0x[b] + 0.5 * dSx);
      if (acc != 0.0) add_at(s, J[2], lz + a, lx + b, 0, acc);
    }
  }
  /* Jx: prefix along x for every z node */
  for (int a = 0; a < nz_; a++) {
    double dSz = S1z[a] - S0z[a], acc = 0.0;
    for (int b = 0; b < nx_; b++) {
      double dSx = S1x[b] - S0x[b];
      acc += cx * dSx * (S0z[a] + 0.5 * dSz);
      if (acc != 0.0) add_at(s, J[0], lz + a, lx + b, 0, acc);
    }
  }
  /* Jy: out-of-plane, the time-averaged shape */
  if (vy != 0.0) {
    for (int a = 0; a < nz_; a++) {
      double dSz = S1z[a] - S0z[a];
      for (int b = 0; b < nx_; b++) {
        double dSx = S1x[b] - S0x[b];
        double wy = S0z[a] * S0x[b] + 0.5 * dSz * S0x[b] + 0.5 * S0z[a] * dSx +
                    dSz * dSx / 3.0;
        if (wy != 0.0) add_at(s, J[1], lz + a, lx + b, 0, cy * wy);
      }
    }
  }
}

static double wmix(double S0a, double dSa, double S0b, double dSb) {
  return S0a * S0b + 0.5 * dSa * S0b + 0.5 * S0a * dSb + dSa * dSb / 3.0;
}

static void deposit_3d(const orc_sim* s, double* const* J, double q, double w, xpos z0,
                       xpos x0, xpos y0, xpos z1, xpos x1, xpos y1) {
  const orc_config* c = &s->c;
  int64_t lz, lx, ly;
  int nz_, nx_, ny_;
  double S0z[STN], S1z[STN], S0x[STN], S1x[STN], S0y[STN], S1y[STN];
  shape_row(c->order, z0, z1, &lz, &nz_, S0z, S1z);
  shape_row(c->order, x0, x1, &lx, &nx_, S0x, S1x);
  shape_row(c->order, y0, y1, &ly, &ny_, S0y, S1y);
  double cz = -q * w / (c->dx * c->dy * c->dt);
  double cx = -q * w / (c->dz * c->dy * c->dt);
  double cy = -q * w / (c->dz * c->dx * c->dt);
  for (int b = 0; b < nx_; b++)
    for (int d = 0; d < ny_; d++) {
      double acc = 0.0;
      for (int a = 0; a < nz_; a++) {
        acc += cz * (S1z[a] - S0z[a]) * wmix(S0x[b], S1x[b] - S0x[b], S0y[d], S1y[d] - S0y[d]);
        if (acc != 0.0) add_at(s, J[2], lz + a, lx + b, ly + d, acc);
      }
    }
  for (int a = 0; a < nz_; a++)
    for (int d = 0; d < ny_; d++) {
      double acc = 0.0;
      for (int b = 0; b < nx_; b++) {
        acc += cx * (S1x[b] - S0x[b]) * wmix(S0z[a], S1z[a] - S0z[a], S0y[d], S1y[d] - S0y[d]);
        if (acc != 0.0) add_at(s, J[0], lz + a, lx + b, ly + d, acc);
      }
    }
  for (int a = 0; a < nz_; a++)
    for (int b = 0; b < nx_; b++) {
      double acc = 0.0;
      for (int d = 0; d < ny_; d++) {
        acc += cy * (S1y[d] - S0y[d]) * wmix(S0z[a], S1z[a] - S0z[a], S0x[b], S1x[b] - S0x[b]);
        if (acc != 0.0) add_at(s, J[1], lz + a, lx + b, ly + d, acc);
      }
    }
}

/* Charge density on the integer lattice (diagnostics): rho += q w S S [S] / dV */
static void deposit_rho(orc_sim* s, double* R, double q, double w, xpos z, xpos x, xpos y) {
  const orc_config* c = &s->c;
  double dV = c->dz * c->dx * (c->dim == 3 ? c->dy : 1.0);
  int64_t i0 = ifloorx(z) - 2, j0 = ifloorx(x) - 2, k0 = ifloorx(y) - 2;
  double lz = (double)(z - (xpos)i0), lx = (double)(x - (xpos)j0), ly = (double)(y - (xpos)k0);
  for (int a = 0; a < 6; a++) {
    double wz = orc_shape(c->order, lz - (double)a);
    if (wz == 0.0) continue;
    for (int b = 0; b < 6; b++) {
      double wx = orc_shape(c->order, lx - (double)b);
      if (wx == 0.0) continue;
      if (c->dim == 2) {
        add_at(s, R, i0 + a, j0 + b, 0, q * w * wz * wx / dV);
      } else {
        for (int d = 0; d < 6; d++) {
          double wy = orc_shape(c->order, ly - (double)d);
          if (wy != 0.0) add_at(s, R, i0 + a, j0 + b, k0 + d, q * w * wz * wx * wy / dV);
        }
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Digital filter (section "Mitigation of a numerical instability": filtering */
/* of short wavelengths as the lever against the instability).  Per axis:    */
/* N passes of (1/4, 1/2, 1/4), then (-N/4, 1 + N/2, -N/4) if compensating.   */
/* Values outside a non-periodic z domain count as zero.                      */
/* ------------------------------------------------------------------------ */
static void zero_outside(orc_sim* s, double* A, double sz) {
  const orc_config* c = &s->c;
  if (c->zbc == 0) return;
  for (int64_t i = -G_ROWS; i <= c->nz + G_ROWS; i++) {
    if (in_domain(s, sz, i)) continue;
    memset(A + (i + G_ROWS) * s->plane, 0, sizeof(double) * (size_t)s->plane);
  }
}

static void filter_pass(orc_sim* s, double* A, double sz, int axis, double a, double b) {
  const orc_config* c = &s->c;
  int64_t total = (int64_t)s->nzs * s->plane;
  double* T = (double*)malloc(sizeof(double) * (size_t)total);
  memcpy(T, A, sizeof(double) * (size_t)total);
  int ny = s->nyy;
  int nt = s->nthreads > 1 ? s->nthreads : 1;
  (void)nt;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static)
#endif
  for (int64_t i = row_lo(s, sz); i <= row_hi(s, sz); i++)
    for (int64_t j = 0; j < c->nx; j++)
      for (int64_t k = 0; k < ny; k++) {
        int64_t di = axis == 0, dj = axis == 1, dk = axis == 2;
        double vm, vp;
        if (axis == 0 && c->zbc != 0) {
          vm = in_domain(s, sz, i - 1) ? T[node(s, i - 1, j, k)] : 0.0;
          vp = in_domain(s, sz, i + 1) ? T[node(s, i + 1, j, k)] : 0.0;
        } else {
          vm = T[node(s, i - di, j - dj, k - dk)];
          vp = T[node(s, i + di, j + dj, k + dk)];
        }
        A[node(s, i, j, k)] = a * vm + b * T[node(s, i, j, k)] + a * vp;
      }
  free(T);
}

static void apply_filter(orc_sim* s, double* A, double sz) {
  const orc_config* c = &s->c;
  zero_outside(s, A, sz);
  int naxes = c->dim == 3 ? 3 : 2;
  for (int axis = 0; axis < naxes; axis++) {
    for (int p = 0; p < c->filter_passes; p++) filter_pass(s, A, sz, axis, 0.25, 0.5);
    if (c->filter_compensate && c->filter_passes > 0) {
      double N = (double)c->filter_passes;
      filter_pass(s, A, sz, axis, -0.25 * N, 1.0 + 0.5 * N);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Yee FDTD (Yee 1966) with B at integer times through two half steps:       */
/*   B <- B - (dt/2) curl E;  E <- E + dt (curl B - J);  B <- B - (dt/2) curl E*/
/* ------------------------------------------------------------------------ */
#define FX(comp, i, j, k) fget(s, comp, i, j, k)

static void yee_b(orc_sim* s, double h) {
  const orc_config* c = &s->c;
  int d3 = c->dim == 3;
  double idz = 1.0 / c->dz, idx = 1.0 / c->dx, idy = d3 ? 1.0 / c->dy : 0.0;
  int nt = s->nthreads > 1 ? s->nthreads : 1;
  (void)nt;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static)
#endif
  for (int64_t j = 0; j < c->nx; j++)
    for (int64_t k = 0; k < s->nyy; k++) {
      for (int64_t i = 0; i <= row_hi(s, 0.5); i++) {
        double dEz_dy = d3 ? (FX(ORC_EZ, i, j, k + 1) - FX(ORC_EZ, i, j, k)) * idy : 0.0;
        s->F[ORC_BX][node(s, i, j, k)] +=
            h * ((FX(ORC_EY, i + 1, j, k) - FX(ORC_EY, i, j, k)) * idz - dEz_dy);
        s->F[ORC_BY][node(s, i, j, k)] +=
            h * ((FX(ORC_EZ, i, j + 1, k) - FX(ORC_EZ, i, j, k)) * idx -
                 (FX(ORC_EX, i + 1, j, k) - FX(ORC_EX, i, j, k)) * idz);
      }
      for (int64_t i = 0; i <= row_hi(s, 0.0); i++) {
        double dEx_dy = d3 ? (FX(ORC_EX, i, j, k + 1) - FX(ORC_EX, i, j, k)) * idy : 0.0;
        s->F[ORC_BZ][node(s, i, j, k)] +=
            h * (dEx_dy - (FX(ORC_EY, i, j + 1, k) - FX(ORC_EY, i, j, k)) * idx);
      }
    }
}

static void yee_e(orc_sim* s, double h) {
  const orc_config* c = &s->c;
  int d3 = c->dim == 3;
  int64_t nz = c->nz;
  double idz = 1.0 / c->dz, idx = 1.0 / c->dx, idy = d3 ? 1.0 / c->dy : 0.0;
  int mur = c->zbc != 0;
  /* old tangential E on the boundary planes and their neighbours, for Mur */
  int64_t plane = s->plane;
  double* old = NULL;
  if (mur) {
    old = (double*)malloc(sizeof(double) * (size_t)(8 * plane));
    int rows[4] = {0, 1, (int)nz - 1, (int)nz};
    for (int r = 0; r < 4; r++) {
      memcpy(old + (2 * r + 0) * plane, s->F[ORC_EX] + (rows[r] + G_ROWS) * plane,
             sizeof(double) * (size_t)plane);
      memcpy(old + (2 * r + 1) * plane, s->F[ORC_EY] + (rows[r] + G_ROWS) * plane,
             sizeof(double) * (size_t)plane);
    }
  }
  int64_t tlo = mur ? 1 : 0, thi = mur ? nz - 1 : nz - 1;
  int nt = s->nthreads > 1 ? s->nthreads : 1;
  (void)nt;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static)
#endif
  for (int64_t j = 0; j < c->nx; j++)
    for (int64_t k = 0; k < s->nyy; k++) {
      for (int64_t i = tlo; i <= thi; i++) {
        double dBz_dy = d3 ? (FX(ORC_BZ, i, j, k) - FX(ORC_BZ, i, j, k - 1)) * idy : 0.0;
        s->F[ORC_EX][node(s, i, j, k)] +=
            h * (dBz_dy - (FX(ORC_BY, i, j, k) - FX(ORC_BY, i - 1, j, k)) * idz -
                 FX(ORC_JX, i, j, k));
        s->F[ORC_EY][node(s, i, j, k)] +=
            h * ((FX(ORC_BX, i, j, k) - FX(ORC_BX, i - 1, j, k)) * idz -
                 (FX(ORC_BZ, i, j, k) - FX(ORC_BZ, i, j - 1, k)) * idx - FX(ORC_JY, i, j, k));
      }
      for (int64_t i = 0; i <= row_hi(s, 0.5); i++) {
        double dBx_dy = d3 ? (FX(ORC_BX, i, j, k) - FX(ORC_BX, i, j, k - 1)) * idy : 0.0;
        s->F[ORC_EZ][node(s, i, j, k)] +=
            h * ((FX(ORC_BY, i, j, k) - FX(ORC_BY, i, j - 1, k)) * idx - dBx_dy -
                 FX(ORC_JZ, i, j, k));
      }
    }
  if (mur) {
    /* first-order Mur, normal incidence: E0' = E1 + m (E1' - E0), m = (dt-dz)/(dt+dz) */
    double m = (c->dt - c->dz) / (c->dt + c->dz);
    for (int comp = 0; comp < 2; comp++) {
      int f = comp == 0 ? ORC_EX : ORC_EY;
      double* o0 = old + (0 + comp) * plane;   /* row 0 */
      double* o1 = old + (2 + comp) * plane;   /* row 1 */
      double* o2 = old + (4 + comp) * plane;   /* row nz-1 */
      double* o3 = old + (6 + comp) * plane;   /* row nz */
      double* n0 = s->F[f] + (0 + G_ROWS) * plane;
      double* n1 = s->F[f] + (1 + G_ROWS) * plane;
      double* n2 = s->F[f] + (nz - 1 + G_ROWS) * plane;
      double* n3 = s->F[f] + (nz + G_ROWS) * plane;
      for (int64_t q = 0; q < plane; q++) {
        n0[q] = o1[q] + m * (n1[q] - o0[q]);
        n3[q] = o2[q] + m * (n2[q] - o3[q]);
      }
    }
    free(old);
  }
}

/* ------------------------------------------------------------------------ */
/* Laser: lab-frame vector potential of a Gaussian pulse (paraxial Gaussian  */
/* beam, y polarised, along +z), evaluated on the calculation frame's t' = 0 */
/* hyperplane, i.e. at lab (t, z) = (gamma beta z', gamma z') -- the frame   */
/* change as a hyperbolic rotation (section "Effect of the hyperbolic        */
/* rotation").  A_y is a transverse component of the four-potential and so   */
/* is invariant; Ey' = -dA/dt' = gamma (1-beta) dA/dxi - gamma beta dA/dzeta.*/
/* ------------------------------------------------------------------------ */
static void lab_potential(const orc_laser* L, int dim, double xi, double zeta, double x,
                          double y, double* A, double* dxi, double* dzeta) {
  double G = 1.0, Gp = 0.0;
  if (L->L > 0.0) {
    if (fabs(xi) > 4.0 * L->L) {
      *A = *dxi = *dzeta = 0.0;
      return;
    }
    double l2 = L->L * L->L;
    G = exp(-xi * xi / l2);
    Gp = -2.0 * xi / l2 * G;
  }
  double complex U = 1.0, dU = 0.0;
  double r2 = dim == 3 ? x * x + y * y : x * x;
  if (L->w0 > 0.0) {
    if (L->collimated) {
      U = exp(-r2 / (L->w0 * L->w0));
    } else {
      /* 2 i dU/dzeta + lap_perp U = 0 solved by q(zeta) = zeta - i zR */
      double zR = 0.5 * L->w0 * L->w0;
      double complex q = zeta - I * zR, q0 = -I * zR;
      double complex ex = cexp(I * r2 / (2.0 * q));
      if (dim == 2) {
        U = csqrt(q0 / q) * ex;
        dU = U * (-1.0 / (2.0 * q) - I * r2 / (2.0 * q * q));
      } else {
        U = (q0 / q) * ex;
        dU = U * (-1.0 / q - I * r2 / (2.0 * q * q));
      }
    }
  }
  double complex ph = cexp(I * (xi + L->phase));
  *A = L->a0 * G * cimag(U * ph);
  *dxi = L->a0 * (Gp * cimag(U * ph) + G * creal(U * ph));
  *dzeta = L->a0 * G * cimag(dU * ph);
}

void orc_laser_eval(const orc_laser* L, int32_t dim, double gamma_b, double tp, double zp,
                    double x, double y, double* A, double* Ey) {
  double beta = orc_beta_of_gamma(gamma_b);
  double omb = orc_one_minus_beta(gamma_b);
  /* lab event: t = gamma (t' + beta z'), z = gamma (z' + beta t');
   * z - t - zc = gamma (1 - beta) (z' - t') - zc */
  double xi = gamma_b * omb * (zp - tp) - L->z_center;
  double zeta = gamma_b * (zp + beta * tp) - L->z_focus;
  double a, dxi, dzeta;
  lab_potential(L, dim, xi, zeta, x, y, &a, &dxi, &dzeta);
  *A = a;
  *Ey = gamma_b * omb * dxi - gamma_b * beta * dzeta;
}

static void init_laser(orc_sim* s, const orc_laser* L) {
  const orc_config* c = &s->c;
  int d3 = c->dim == 3;
  double xa = 0.5 * c->nx * c->dx, ya = d3 ? 0.5 * c->ny * c->dy : 0.0;
  double Lz = c->nz * c->dz, Lx = c->nx * c->dx, Ly = d3 ? c->ny * c->dy : 0.0;
  int ihi = row_hi(s, 0.0);
  int64_t total = (int64_t)s->nzs * s->plane;
  double* A = (double*)calloc((size_t)total, sizeof(double));
  int my = d3 ? L->images_y : 0;
  int nt = s->nthreads > 1 ? s->nthreads : 1;
  (void)nt;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(dynamic, 4)
#endif
  for (int64_t i = 0; i <= ihi; i++)
    for (int64_t j = 0; j < c->nx; j++)
      for (int64_t k = 0; k < s->nyy; k++) {
        double zp = (double)i * c->dz;
        double x = (double)j * c->dx - xa;
        double y = d3 ? ((double)k + 0.5) * c->dy - ya : 0.0;
        double As = 0.0, Es = 0.0;
        for (int mz = -L->images_z; mz <= L->images_z; mz++)
          for (int mx = -L->images_x; mx <= L->images_x; mx++)
            for (int mm = -my; mm <= my; mm++) {
              double a, e;
              orc_laser_eval(L, c->dim, c->gamma_b, 0.0, zp + mz * Lz, x + mx * Lx,
                             y + mm * Ly, &a, &e);
              As += a;
              Es += e;
            }
        A[node(s, i, j, k)] = As;
        s->F[ORC_EY][node(s, i, j, k)] += Es;
      }
  /* B = curl_h (0, A_y, 0): Bx = -dA/dz at (i+1/2, j[, k+1/2]), Bz = dA/dx at (i, j+1/2[, k+1/2]) */
  for (int64_t j = 0; j < c->nx; j++)
    for (int64_t k = 0; k < s->nyy; k++) {
      for (int64_t i = 0; i <= row_hi(s, 0.5); i++) {
        int64_t n1 = node(s, i + 1, j, k);
        double a1 = n1 < 0 ? 0.0 : A[n1];
        s->F[ORC_BX][node(s, i, j, k)] += -(a1 - A[node(s, i, j, k)]) / c->dz;
      }
      for (int64_t i = 0; i <= ihi; i++)
        s->F[ORC_BZ][node(s, i, j, k)] +=
            (A[node(s, i, j + 1, k)] - A[node(s, i, j, k)]) / c->dx;
    }
  /* 3D: Ez from discrete Gauss div E = 0 integrated from the low z end */
  if (d3) {
    for (int64_t j = 0; j < c->nx; j++)
      for (int64_t k = 0; k < c->ny; k++) {
        double acc = 0.0;
        for (int64_t i = 0; i <= row_hi(s, 0.5); i++) {
          acc -= c->dz * (FX(ORC_EY, i, j, k) - FX(ORC_EY, i, j, k - 1)) / c->dy;
          s->F[ORC_EZ][node(s, i, j, k)] += acc;
        }
      }
  }
  free(A);
}

/* ------------------------------------------------------------------------ */
/* Plasma: a lab-rest plasma seen from the boosted frame has density         */
/* gamma_b n and momentum u_b = -gamma_b beta_b along z.  Particles sit on   */
/* a lattice rigid in the calculation frame; column k occupies co-moving     */
/* cells [k, k+1).  Lab birth coordinate z_lab = gamma_b (k + r_z) dz.       */
/* ------------------------------------------------------------------------ */
/* Piecewise-linear lab density through the knots (z_m, n_m), zero outside
 * [z_0, z_last].  The bracketing segment [z_m, z_m+1] is found by bisection
 * on the increasing knot positions; the value is the barycentric mix
 * n_m (z_m+1 - z) / h + n_m+1 (z - z_m) / h with h = z_m+1 - z_m. */
static double lab_density(const orc_sim* s, double zl) {
  if (s->nknots < 2) return s->n_uniform;
  const double* kz = s->kz;
  int last = s->nknots - 1;
  if (!(zl >= kz[0] && zl <= kz[last])) return 0.0;
  int lo = 0, hi = last; /* invariant: kz[lo] <= zl <= kz[hi] */
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (kz[mid] <= zl) lo = mid;
    else hi = mid;
  }
  double h = kz[hi] - kz[lo];
  double a = (kz[hi] - zl) / h, b = (zl - kz[lo]) / h;
  return s->kn[lo] * a + s->kn[hi] * b;
}

/* Plasma channel: the lab density times 1 + depth r^2 / radius^2, r the
 * distance of the birth position from the laser axis (the box centre, x in
 * 2D, x and y in 3D).  A parabolic channel of depth dn / n at r = w0 guides a
 * Gaussian beam of waist w0 when dn / n_c = 4 / (k0 w0)^2 (paraxial mode of a
 * parabolic index profile, applied per transverse axis).  x, y in cells. */
static double channel_factor(const orc_sim* s, double x, double y) {
  const orc_config* c = &s->c;
  if (s->ch_depth == 0.0) return 1.0;
  double rx = (x - 0.5 * (double)c->nx) * c->dx;
  double ry = c->dim == 3 ? (y - 0.5 * (double)c->ny) * c->dy : 0.0;
  double r2 = rx * rx + ry * ry;
  return 1.0 + s->ch_depth * (r2 / (s->ch_radius * s->ch_radius));
}

double orc_lab_density(const orc_sim* s, double z_lab) { return lab_density(s, z_lab); }

double orc_channel_factor(const orc_sim* s, double x, double y) {
  return channel_factor(s, x, y);
}

static void grow(orc_sim* s, int64_t need) {
  if (need <= s->cap) return;
  int64_t nc = s->cap ? s->cap : 1024;
  while (nc < need) nc *= 2;
  xpos** pos[6] = {&s->ze, &s->xe, &s->ye, &s->zi, &s->xi, &s->yi};
  for (int a = 0; a < 6; a++) *pos[a] = (xpos*)realloc(*pos[a], sizeof(xpos) * (size_t)nc);
  double** arrs[4] = {&s->uz, &s->ux, &s->uy, &s->w};
  for (int a = 0; a < 4; a++) *arrs[a] = (double*)realloc(*arrs[a], sizeof(double) * (size_t)nc);
  s->id = (int64_t*)realloc(s->id, sizeof(int64_t) * (size_t)nc);
  s->cap = nc;
}

static void store_pair(orc_sim* s, xpos ze, xpos xe, xpos ye, double uz, double ux, double uy,
                       xpos zi, xpos xi, xpos yi, double w, int64_t id) {
  grow(s, s->np + 1);
  int64_t p = s->np++;
  s->ze[p] = ze; s->xe[p] = xe; s->ye[p] = ye;
  s->uz[p] = uz; s->ux[p] = ux; s->uy[p] = uy;
  s->zi[p] = zi; s->xi[p] = xi; s->yi[p] = yi;
  s->w[p] = w; s->id[p] = id;
}

int orc_add_pair(orc_sim* s, double ze, double xe, double ye, double uz, double ux, double uy,
                 double zi, double xi, double yi, double w, int64_t id) {
  store_pair(s, ze, xe, ye, uz, ux, uy, zi, xi, yi, w, id);
  return 0;
}

void orc_clear_particles(orc_sim* s) { s->np = 0; }

/* D = step * s_b + window cells, with s_b = beta_b dt / dz rounded once to
 * FP64 (the step the partners take) and the product formed in extended
 * precision, as the partners' positions accumulate it. */
static xpos drift_cells_x(const orc_sim* s) {
  double bb = orc_beta_of_gamma(s->c.gamma_b);
  double sb = (bb * s->c.dt) / s->c.dz;
  return (xpos)s->step * (xpos)sb + (xpos)s->window_cells;
}
static double drift_cells(const orc_sim* s) { return (double)drift_cells_x(s); }

static void add_column(orc_sim* s, int64_t k, xpos D) {
  const orc_config* c = &s->c;
  int d3 = c->dim == 3;
  double ub = orc_drift_u(c->gamma_b);
  double dV = c->dz * c->dx * (d3 ? c->dy : 1.0);
  for (int64_t l = 0; l < s->nyy; l++)
    for (int64_t j = 0; j < c->nx; j++)
      for (int32_t q = 0; q < c->ppc; q++) {
        double rz = 0.5, rx = 0.5, ry = d3 ? 0.5 : 0.0;
        if (!c->load) {
          rz = orc_cell_offset(c->seed, k, l, j, q, 0, c->nx, s->nyy, c->ppc);
          rx = orc_cell_offset(c->seed, k, l, j, q, 1, c->nx, s->nyy, c->ppc);
          ry = d3 ? orc_cell_offset(c->seed, k, l, j, q, 2, c->nx, s->nyy, c->ppc) : 0.0;
        }
        double zl = c->gamma_b * ((double)k + rz) * c->dz;
        xpos z = ((xpos)k + (xpos)rz) - D;
        double x = (double)j + rx, y = (double)l + ry;
        double w = c->gamma_b * lab_density(s, zl) * channel_factor(s, x, y) * dV / (double)c->ppc;
        int64_t id = ((k * s->nyy + l) * c->nx + j) * c->ppc + q;
        store_pair(s, z, x, y, ub + s->du0[2], s->du0[0], s->du0[1], z, x, y, w, id);
      }
}

/* Continuous injection: column k enters once its low edge k - D is below nz. */
static void inject_due(orc_sim* s) {
  if (!s->has_plasma || s->c.zbc == 0) return;
  xpos D = drift_cells_x(s);
  while ((xpos)s->next_col - D < (xpos)s->c.nz) {
    add_column(s, s->next_col, D);
    s->next_col++;
  }
}

/* ------------------------------------------------------------------------ */
/* Lifecycle                                                                  */
/* ------------------------------------------------------------------------ */
orc_sim* orc_create(const orc_config* cfg) {
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  s->c = *cfg;
  s->nyy = cfg->dim == 3 ? cfg->ny : 1;
  s->nzs = cfg->nz + 2 * G_ROWS + 1;
  s->plane = (int64_t)cfg->nx * s->nyy;
  int64_t total = (int64_t)s->nzs * s->plane;
  for (int a = 0; a < ORC_NCOMP; a++) s->F[a] = (double*)calloc((size_t)total, sizeof(double));
  s->rho = (double*)calloc((size_t)total, sizeof(double));
  s->ant_row = -1;
  return s;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  for (int a = 0; a < ORC_NCOMP; a++) free(s->F[a]);
  free(s->rho);
  xpos* pos[6] = {s->ze, s->xe, s->ye, s->zi, s->xi, s->yi};
  for (int a = 0; a < 6; a++) free(pos[a]);
  double* arrs[4] = {s->uz, s->ux, s->uy, s->w};
  for (int a = 0; a < 4; a++) free(arrs[a]);
  free(s->id);
  free(s->kz);
  free(s->kn);
  orc_set_threads(s, 1);
  free(s);
}

int orc_init(orc_sim* s, const orc_density* dens, const orc_laser* laser, int32_t fill) {
  const orc_config* c = &s->c;
  int64_t total = (int64_t)s->nzs * s->plane;
  for (int a = 0; a < ORC_NCOMP; a++) memset(s->F[a], 0, sizeof(double) * (size_t)total);
  s->np = 0;
  s->step = 0;
  s->window_cells = 0.0;
  s->next_col = 0;
  s->has_plasma = dens != NULL;
  free(s->kz);
  free(s->kn);
  s->kz = s->kn = NULL;
  s->nknots = 0;
  s->du0[0] = s->du0[1] = s->du0[2] = 0.0;
  s->ch_depth = 0.0;
  s->ch_radius = 1.0;
  if (dens) {
    if (!(dens->channel_depth >= 0.0) || (dens->channel_depth > 0.0 && !(dens->channel_radius > 0.0)))
      return -1;
    s->ch_depth = dens->channel_depth;
    if (dens->channel_depth > 0.0) s->ch_radius = dens->channel_radius;
    for (int a = 0; a < 3; a++) s->du0[a] = dens->du[a];
    s->n_uniform = dens->n_uniform;
    s->nknots = dens->nknots;
    if (dens->nknots >= 2) {
      s->kz = (double*)malloc(sizeof(double) * (size_t)dens->nknots);
      s->kn = (double*)malloc(sizeof(double) * (size_t)dens->nknots);
      memcpy(s->kz, dens->z_lab, sizeof(double) * (size_t)dens->nknots);
      memcpy(s->kn, dens->n, sizeof(double) * (size_t)dens->nknots);
    }
  }
  if (laser) init_laser(s, laser);
  if (dens && fill) {
    for (int64_t k = 0; k < c->nz; k++) add_column(s, k, 0.0);
    s->next_col = c->nz;
  }
  return 0;
}

int orc_window_shift(orc_sim* s, int32_t n) {
  const orc_config* c = &s->c;
  if (n == 0) return 0;
  if (c->zbc == 0) return -1;
  int64_t plane = s->plane;
  for (int a = 0; a < ORC_NCOMP; a++) {
    double* T = (double*)calloc((size_t)(s->nzs * plane), sizeof(double));
    for (int64_t i = -G_ROWS; i <= c->nz + G_ROWS; i++) {
      int64_t src = i + n;
      if (src < -G_ROWS || src > c->nz + G_ROWS) continue;
      memcpy(T + (i + G_ROWS) * plane, s->F[a] + (src + G_ROWS) * plane,
             sizeof(double) * (size_t)plane);
    }
    memcpy(s->F[a], T, sizeof(double) * (size_t)(s->nzs * plane));
    free(T);
    zero_outside(s, s->F[a], SIG[a][0]);
  }
  for (int64_t p = 0; p < s->np; p++) {
    s->ze[p] -= n;
    s->zi[p] -= n;
  }
  s->window_cells += n;
  return 0;
}

/* Threads of the particle loop: the count set by orc_set_threads (1 by
 * default), but no more than one per 4096 pairs; the per-thread current
 * buffers are allocated on first use and kept. */
static int orc_threads_for(orc_sim* s) {
  int nt = s->nthreads > 1 ? s->nthreads : 1;
  int64_t lim = s->np / 4096;
  if (lim < 1) lim = 1;
  if (nt > lim) nt = (int)lim;
  if (nt > 1 && !s->tJ) {
    int64_t total = (int64_t)s->nzs * s->plane;
    s->tJ = (double**)calloc((size_t)(3 * (s->nthreads - 1)), sizeof(double*));
    for (int t = 0; t < 3 * (s->nthreads - 1); t++)
      s->tJ[t] = (double*)malloc(sizeof(double) * (size_t)total);
  }
  return nt;
}

int orc_set_threads(orc_sim* s, int32_t n) {
  if (n < 1) return -1;
#ifndef _OPENMP
  if (n > 1) return -1;
#endif
  if (s->tJ) {
    for (int t = 0; t < 3 * (s->nthreads - 1); t++) free(s->tJ[t]);
    free(s->tJ);
    s->tJ = NULL;
  }
  s->nthreads = n;
  return 0;
}

int32_t orc_max_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

/* One full step: inject -> (gather, Boris, move, deposit) per electron,
 * rigid drift + deposit per ion partner -> filter J -> Yee -> removal. */
/* Laser antenna.  A sheet of current K (per unit transverse area) in the plane
 * z = z_a radiates E_y = -K/2 on both sides in 1D vacuum (the jump of B_x
 * across the sheet is K, split evenly between the two outgoing waves).  A
 * sheet on one row of the grid carries K = J_y dz, so the current
 * J_y = -2 E_target / dz, applied over the step n -> n+1 (time-centred at
 * t' = (n + 1/2) dt), emits the target field E_y'(t', z_a, x[, y]) of the
 * laser into both directions.  The target is the boosted laser of init (its
 * lab potential evaluated at the boosted event), with the same transverse
 * images; the row is fixed on the grid and z_a = (row + window) dz.  The
 * current is added after the filter (the source is not smoothed). */
static void antenna_source(orc_sim* s) {
  const orc_config* c = &s->c;
  const orc_laser* L = &s->ant;
  int d3 = c->dim == 3;
  double tp = ((double)s->step + 0.5) * c->dt;
  double zp = ((double)s->ant_row + s->window_cells) * c->dz;
  double xa = 0.5 * c->nx * c->dx, ya = d3 ? 0.5 * c->ny * c->dy : 0.0;
  double Lx = c->nx * c->dx, Ly = d3 ? c->ny * c->dy : 0.0;
  int my = d3 ? L->images_y : 0;
  for (int64_t j = 0; j < c->nx; j++)
    for (int64_t k = 0; k < s->nyy; k++) {
      double x = (double)j * c->dx - xa;
      double y = d3 ? ((double)k + 0.5) * c->dy - ya : 0.0;
      double Es = 0.0;
      for (int mx = -L->images_x; mx <= L->images_x; mx++)
        for (int mm = -my; mm <= my; mm++) {
          double a, e;
          orc_laser_eval(L, c->dim, c->gamma_b, tp, zp, x + mx * Lx, y + mm * Ly, &a, &e);
          Es += e;
        }
      s->F[ORC_JY][node(s, s->ant_row, j, k)] += -2.0 * Es / c->dz;
    }
}

int orc_set_antenna(orc_sim* s, const orc_laser* laser, int32_t row) {
  if (!laser || row < 0) {
    s->ant_row = -1;
    return 0;
  }
  if (row < 1 || row > s->c.nz - 1) return -1;
  s->ant = *laser;
  s->ant_row = row;
  return 0;
}

int orc_step(orc_sim* s, int32_t nsteps) {
  const orc_config* c = &s->c;
  int d3 = c->dim == 3;
  int64_t total = (int64_t)s->nzs * s->plane;
  double bb = orc_beta_of_gamma(c->gamma_b);
  double sb = (bb * c->dt) / c->dz;
  for (int32_t it = 0; it < nsteps; it++) {
    inject_due(s);
    for (int a = ORC_JX; a <= ORC_JZ; a++) memset(s->F[a], 0, sizeof(double) * (size_t)total);
    /* Particles are independent within a step: each thread pushes a share of
     * them and deposits into its own current buffer; the buffers are summed
     * into J afterwards (same sums, another order of addition). */
    int nt = orc_threads_for(s);
    for (int t = 1; t < nt; t++)
      for (int a = 0; a < 3; a++) memset(s->tJ[3 * (t - 1) + a], 0, sizeof(double) * (size_t)total);
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static)
#endif
    for (int64_t p = 0; p < s->np; p++) {
#ifdef _OPENMP
      int th = omp_get_thread_num();
#else
      int th = 0;
#endif
      double* const Jt[3] = {th ? s->tJ[3 * (th - 1) + 0] : s->F[ORC_JX],
                             th ? s->tJ[3 * (th - 1) + 1] : s->F[ORC_JY],
                             th ? s->tJ[3 * (th - 1) + 2] : s->F[ORC_JZ]};
      xpos z0 = s->ze[p], x0 = s->xe[p], y0 = s->ye[p];
      double E[3], B[3];
      E[0] = gather(s, ORC_EX, z0, x0, y0);
      E[1] = gather(s, ORC_EY, z0, x0, y0);
      E[2] = gather(s, ORC_EZ, z0, x0, y0);
      B[0] = gather(s, ORC_BX, z0, x0, y0);
      B[1] = gather(s, ORC_BY, z0, x0, y0);
      B[2] = gather(s, ORC_BZ, z0, x0, y0);
      double u[3] = {s->ux[p], s->uy[p], s->uz[p]};
      orc_boris(-1.0, c->dt, E, B, u);
      double g = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      double vx = u[0] / g, vy = u[1] / g, vz = u[2] / g;
      xpos z1 = z0 + (xpos)(vz * c->dt / c->dz);
      xpos x1 = x0 + (xpos)(vx * c->dt / c->dx);
      xpos y1 = d3 ? y0 + (xpos)(vy * c->dt / c->dy) : y0;
      if (d3) deposit_3d(s, Jt, -1.0, s->w[p], z0, x0, y0, z1, x1, y1);
      else deposit_2d(s, Jt, -1.0, s->w[p], vy, z0, x0, z1, x1);
      s->ux[p] = u[0];
      s->uy[p] = u[1];
      s->uz[p] = u[2];
      s->ze[p] = c->zbc == 0 ? z1 - (xpos)c->nz * (xpos)ifloorx(z1 / (xpos)c->nz) : z1;
      s->xe[p] = x1 - (xpos)c->nx * (xpos)ifloorx(x1 / (xpos)c->nx);
      s->ye[p] = d3 ? y1 - (xpos)c->ny * (xpos)ifloorx(y1 / (xpos)c->ny) : y1;
      if (c->ions && sb != 0.0) {
        xpos zi0 = s->zi[p], zi1 = zi0 - (xpos)sb;
        if (d3) deposit_3d(s, Jt, 1.0, s->w[p], zi0, s->xi[p], s->yi[p], zi1, s->xi[p], s->yi[p]);
        else deposit_2d(s, Jt, 1.0, s->w[p], 0.0, zi0, s->xi[p], zi1, s->xi[p]);
        s->zi[p] = c->zbc == 0 ? zi1 - (xpos)c->nz * (xpos)ifloorx(zi1 / (xpos)c->nz) : zi1;
      }
    }
    for (int t = 1; t < nt; t++)
      for (int a = 0; a < 3; a++) {
        const double* src = s->tJ[3 * (t - 1) + a];
        double* dst = s->F[ORC_JX + a];
        for (int64_t q = 0; q < total; q++) dst[q] += src[q];
      }
    apply_filter(s, s->F[ORC_JX], SIG[ORC_JX][0]);
    apply_filter(s, s->F[ORC_JY], SIG[ORC_JY][0]);
    apply_filter(s, s->F[ORC_JZ], SIG[ORC_JZ][0]);
    if (s->ant_row >= 0) antenna_source(s);
    yee_b(s, 0.5 * c->dt);
    yee_e(s, c->dt);
    yee_b(s, 0.5 * c->dt);
    /* removal: a pair leaves once both members are more than order+1 cells
     * outside [0, nz] along z, where no stencil reaches the grid any more */
    if (c->zbc != 0) {
      double lim = (double)(c->order + 1);
      int64_t q = 0;
      for (int64_t p = 0; p < s->np; p++) {
        int eout = s->ze[p] < -lim || s->ze[p] > (xpos)(c->nz + lim);
        int iout = !c->ions || s->zi[p] < -lim || s->zi[p] > (xpos)(c->nz + lim);
        if (eout && iout) continue;
        if (q != p) {
          s->ze[q] = s->ze[p]; s->xe[q] = s->xe[p]; s->ye[q] = s->ye[p];
          s->uz[q] = s->uz[p]; s->ux[q] = s->ux[p]; s->uy[q] = s->uy[p];
          s->zi[q] = s->zi[p]; s->xi[q] = s->xi[p]; s->yi[q] = s->yi[p];
          s->w[q] = s->w[p]; s->id[q] = s->id[p];
        }
        q++;
      }
      s->np = q;
    }
    s->step++;
    if (c->auto_window && c->zbc != 0) {
      double t = (double)s->step * c->dt;
      double due = floor((c->beta_window * t) / c->dz) - s->window_cells;
      if (due != 0.0) orc_window_shift(s, (int32_t)due);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics (FP64 sums).                                                   */
/* ------------------------------------------------------------------------ */
int orc_diagnostics(orc_sim* s, orc_diag* o, double* lineout) {
  const orc_config* c = &s->c;
  int d3 = c->dim == 3;
  double dV = c->dz * c->dx * (d3 ? c->dy : 1.0);
  int nanf = 0;
  double ue = 0.0, ub = 0.0;
  for (int a = ORC_EX; a <= ORC_BZ; a++) {
    double acc = 0.0;
    for (int64_t i = 0; i <= row_hi(s, SIG[a][0]); i++)
      for (int64_t q = 0; q < s->plane; q++) {
        double v = s->F[a][(i + G_ROWS) * s->plane + q];
        if (!isfinite(v)) nanf = 1;
        acc += v * v;
      }
    if (a <= ORC_EZ) ue += acc;
    else ub += acc;
  }
  o->ue = 0.5 * ue * dV;
  o->ub = 0.5 * ub * dV;
  double gb = c->gamma_b;
  double ukin = 0.0, ukd = 0.0, charge = 0.0;
  for (int64_t p = 0; p < s->np; p++) {
    double u2 = s->ux[p] * s->ux[p] + s->uy[p] * s->uy[p] + s->uz[p] * s->uz[p];
    double g = sqrt(1.0 + u2);
    if (!isfinite(g) || !isfinite((double)s->ze[p]) || !isfinite((double)s->xe[p])) nanf = 1;
    ukin += s->w[p] * (g - 1.0);
    ukd += s->w[p] * (g - gb);
    charge += -s->w[p];
  }
  o->ukin = ukin;
  o->ukin_drift = ukd;
  o->charge = charge;
  o->live = s->np;
  /* on-axis lineout of Ez and the wake amplitude */
  int64_t ja = c->nx / 2, ka = d3 ? c->ny / 2 : 0;
  double amp = 0.0;
  for (int64_t i = 0; i <= row_hi(s, 0.5); i++) {
    double v = FX(ORC_EZ, i, ja, ka);
    if (lineout) lineout[i] = v;
    if (fabs(v) > amp) amp = fabs(v);
  }
  o->wake_amp = amp;
  /* Gauss residual: max |div_h E - F rho| on the integer lattice */
  int64_t total = (int64_t)s->nzs * s->plane;
  memset(s->rho, 0, sizeof(double) * (size_t)total);
  for (int64_t p = 0; p < s->np; p++) {
    deposit_rho(s, s->rho, -1.0, s->w[p], s->ze[p], s->xe[p], s->ye[p]);
    if (c->ions) deposit_rho(s, s->rho, 1.0, s->w[p], s->zi[p], s->xi[p], s->yi[p]);
  }
  apply_filter(s, s->rho, 0.0);
  int64_t b = c->zbc == 0 ? 0 : (int64_t)(c->filter_passes + c->order + 4);
  int64_t ilo = b, ihi = c->zbc == 0 ? c->nz - 1 : c->nz - b;
  double res = 0.0;
  for (int64_t i = ilo; i <= ihi; i++)
    for (int64_t j = 0; j < c->nx; j++)
      for (int64_t k = 0; k < s->nyy; k++) {
        double dv = (FX(ORC_EZ, i, j, k) - FX(ORC_EZ, i - 1, j, k)) / c->dz +
                    (FX(ORC_EX, i, j, k) - FX(ORC_EX, i, j - 1, k)) / c->dx;
        if (d3) dv += (FX(ORC_EY, i, j, k) - FX(ORC_EY, i, j, k - 1)) / c->dy;
        double r = fabs(dv - s->rho[node(s, i, j, k)]);
        if (r > res) res = r;
      }
  o->gauss_res = res;
  o->step = s->step;
  o->t = (double)s->step * c->dt;
  o->window_cells = s->window_cells;
  o->drift_cells = drift_cells(s);
  o->nan_flag = nanf;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* State access                                                               */
/* ------------------------------------------------------------------------ */
int orc_filter_field(orc_sim* s, int32_t comp) {
  if (comp < 0 || comp >= ORC_NCOMP) return -1;
  apply_filter(s, s->F[comp], SIG[comp][0]);
  return 0;
}

int64_t orc_field_size(const orc_sim* s) { return (int64_t)(s->c.nz + 1) * s->plane; }

int orc_get_field(const orc_sim* s, int32_t comp, double* out) {
  if (comp < 0 || comp >= ORC_NCOMP) return -1;
  memcpy(out, s->F[comp] + G_ROWS * s->plane,
         sizeof(double) * (size_t)((s->c.nz + 1) * s->plane));
  return 0;
}

int orc_set_field(orc_sim* s, int32_t comp, const double* in) {
  if (comp < 0 || comp >= ORC_NCOMP) return -1;
  memcpy(s->F[comp] + G_ROWS * s->plane, in,
         sizeof(double) * (size_t)((s->c.nz + 1) * s->plane));
  if (s->c.zbc == 0) /* row nz does not exist in a periodic box */
    memset(s->F[comp] + (G_ROWS + s->c.nz) * s->plane, 0, sizeof(double) * (size_t)s->plane);
  zero_outside(s, s->F[comp], SIG[comp][0]);
  return 0;
}

int64_t orc_num_pairs(const orc_sim* s) { return s->np; }

int orc_get_particles(const orc_sim* s, double* ze, double* xe, double* ye, double* uz,
                      double* ux, double* uy, double* zi, double* w, int64_t* id) {
  size_t nb = sizeof(double) * (size_t)s->np;
  for (int64_t p = 0; p < s->np; p++) {
    if (ze) ze[p] = (double)s->ze[p];
    if (xe) xe[p] = (double)s->xe[p];
    if (ye) ye[p] = (double)s->ye[p];
    if (zi) zi[p] = (double)s->zi[p];
  }
  if (uz) memcpy(uz, s->uz, nb);
  if (ux) memcpy(ux, s->ux, nb);
  if (uy) memcpy(uy, s->uy, nb);
  if (w) memcpy(w, s->w, nb);
  if (id) memcpy(id, s->id, sizeof(int64_t) * (size_t)s->np);
  return 0;
}

/* Co-moving tile-major key: the electron's co-moving cell (z + D, x[, y])
 * is clamped into the tile rows [tz_min*tz, (tz_min+ntz)*tz) along z, then
 * key = ((tile_z * ntx + tile_x) * nty + tile_y) * (tz*tx*ty)
 *       + (lz * tx + lx) * ty + ly. */
int orc_sort_keys(const orc_sim* s, int32_t tz, int32_t tx, int32_t ty, int64_t tz_min,
                  int32_t ntz, int32_t* key, int32_t* id) {
  const orc_config* c = &s->c;
  int d3 = c->dim == 3;
  if (!d3) ty = 1;
  int64_t ntx = c->nx / tx, nty = d3 ? c->ny / ty : 1;
  xpos D = drift_cells_x(s);
  for (int64_t p = 0; p < s->np; p++) {
    int64_t kz = ifloorx(s->ze[p] + D);
    if (c->zbc == 0) kz = wrapi(kz, c->nz);
    int64_t kx = wrapi(ifloorx(s->xe[p]), c->nx);
    int64_t ky = d3 ? wrapi(ifloorx(s->ye[p]), c->ny) : 0;
    int64_t rz = kz - tz_min * tz;
    if (rz < 0) rz = 0;
    if (rz >= (int64_t)ntz * tz) rz = (int64_t)ntz * tz - 1;
    int64_t tile = ((rz / tz) * ntx + kx / tx) * nty + ky / ty;
    int64_t loc = ((rz % tz) * tx + kx % tx) * ty + ky % ty;
    key[p] = (int32_t)(tile * (int64_t)tz * tx * ty + loc);
    id[p] = (int32_t)s->id[p];
  }
  return 0;
}
