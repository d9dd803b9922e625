/*
 * pic_oracle.h -- plain FP64 CPU particle-in-cell oracle.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark call this library. The product path (the HIP
 * library and its Python binding) never links, loads or runs it, and it
 * shares no source with it.
 *
 * What it computes: one explicit electromagnetic particle-in-cell step in a
 * Lorentz-boosted calculation frame, written out in the plainest form:
 * absolute FP64 particle positions in cell units, naive v = u/gamma, explicit
 * ion partner particles, loops over stencils that evaluate the shape function
 * at every candidate node.  The paper (Vay, Geddes, Cormier-Michel, Grote,
 * "Effects of hyperbolic rotation in Minkowski space on the modeling of
 * plasma accelerators in a Lorentz boosted frame") motivates the boosted
 * frame (introduction; section "Effect of the hyperbolic rotation") and the
 * current filtering that keeps the short-wavelength instability in check
 * (section "Mitigation of a numerical instability"), but it prints no
 * numerical scheme: it says the techniques are described elsewhere.  The
 * steps below are the textbook methods the method is built from:
 *   gather (momentum-conserving, same shape as the deposit)
 *   relativistic Boris push (Boris 1970)
 *   charge-conserving deposit (Esirkepov 2001)
 *   N binomial (1/4,1/2,1/4) passes + optional (-N/4,1+N/2,-N/4) compensation
 *   Yee FDTD with B split into two half steps, first-order Mur at the z ends
 * Units: time 1/omega0, length c/omega0, momentum u = gamma*beta, E in
 * m c omega0/e, B in m omega0/e, density in n_crit, electron q = -1, m = 1.
 *
 * Parity unpinned: nothing here is unpinned at the primitive level; the
 * nonlinear wake amplitude of a full boosted run has no closed form and is
 * compared only against this oracle.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Field component numbering (shared meaning with every array below). */
enum { ORC_EX = 0, ORC_EY, ORC_EZ, ORC_BX, ORC_BY, ORC_BZ, ORC_JX, ORC_JY, ORC_JZ,
       ORC_NCOMP };

typedef struct orc_config {
  int32_t dim;               /* 2: plane (z, x), y invariant; 3: (z, x, y) */
  int32_t nz, nx, ny;        /* cells per axis; ny ignored for dim 2 */
  double dz, dx, dy;         /* cell sizes [c/omega0] */
  double dt;                 /* time step [1/omega0] */
  int32_t order;             /* particle shape: 1 linear, 2 quadratic */
  int32_t filter_passes;     /* N */
  int32_t filter_compensate; /* 0/1 */
  int32_t zbc;               /* 0 periodic z, 1 Mur on tangential E at z ends */
  int32_t ppc;               /* particles per lattice cell */
  uint64_t seed;             /* counter-RNG key for in-cell positions */
  double gamma_b;            /* Lorentz factor of the calculation frame */
  double beta_window;        /* window speed (+z) in the calculation frame */
  int32_t auto_window;       /* 1: shift after each step per the schedule */
  int32_t ions;              /* 1: every electron has a co-located ion partner */
  int32_t load;              /* 0: SplitMix64 in-cell offsets; 1: every slot at the cell centre */
  int32_t gather;            /* 0: momentum-conserving (every axis with the deposit's
                                shape); 1: energy-conserving (Galerkin): along each
                                axis on which a component sits at half-integer
                                nodes, the shape of one order lower */
} orc_config;

typedef struct orc_density {
  double n_uniform;          /* lab density [n_crit] when nknots == 0 */
  int32_t nknots;            /* >= 2: piecewise-linear through knots, 0 outside */
  const double* z_lab;       /* knot positions, lab frame [c/omega0], increasing */
  const double* n;           /* knot densities [n_crit] */
  double du[3];              /* momentum added to every electron at birth (x, y, z) */
  double channel_depth;      /* transverse profile 1 + depth r^2 / radius^2 about the */
  double channel_radius;     /* laser axis (a plasma channel); depth 0: none          */
} orc_density;

typedef struct orc_laser {
  double a0;                 /* peak normalised vector potential */
  double w0;                 /* 1/e field waist at focus; <= 0: plane in x (and y) */
  double L;                  /* 1/e half-length of the field envelope; <= 0: none */
  double z_center;           /* lab pulse centre at lab t = 0 */
  double z_focus;            /* lab focal plane */
  double phase;              /* carrier phase phi0 */
  int32_t collimated;        /* 1: drop the diffraction (zeta) dependence */
  int32_t images_z, images_x, images_y; /* periodisation: sum over +-images */
} orc_laser;

typedef struct orc_diag {
  int64_t step;
  double t;                  /* calculation-frame time */
  double window_cells;       /* total window displacement [cells] */
  double drift_cells;        /* D = n*beta_b*dt/dz + window_cells */
  double ue, ub;             /* field energies 1/2 sum F^2 dV */
  double ukin;               /* sum over electrons w (gamma - 1) */
  double ukin_drift;         /* sum over electrons w (gamma - gamma_b) */
  double wake_amp;           /* max |Ez| on the axis row */
  double gauss_res;          /* max |div E - F rho| over checked nodes */
  double charge;             /* sum over electrons q w */
  int64_t live;              /* live electrons */
  int32_t nan_flag;
} orc_diag;

typedef struct orc_sim orc_sim;

/* ---- boost helper (independent FP64 copy) ---- */
double orc_beta_of_gamma(double gamma);
double orc_one_minus_beta(double gamma);          /* 1 - beta, cancellation-free */
double orc_drift_u(double gamma_b);               /* u_b = -gamma_b beta_b */
double orc_group_gamma(double n_lab);             /* gamma_g = 1/sqrt(n) (cold, 1D) */
double orc_boosted_group_beta(double gamma_b, double n_lab);
double orc_boosted_dz(double gamma_b, double lambda0, double cells_per_wavelength);
double orc_yee_dt(int32_t dim, double dz, double dx, double dy, double cfl);
double orc_depletion_length(double n_lab);        /* lambda_p^3 / (2 lambda0^2) */

/* ---- primitives ---- */
uint64_t orc_splitmix64(uint64_t seed, uint64_t n);  /* n-th output, n >= 1 */
double orc_cell_offset(uint64_t seed, int64_t k, int64_t l, int64_t j, int32_t s,
                       int32_t axis, int32_t nx, int32_t nyy, int32_t ppc);
double orc_shape(int32_t order, double d);
void orc_boris(double q, double dt, const double E[3], const double B[3], double u[3]);
/* Stable sort of (key, id) pairs: perm[d] = source index of destination d. */
void orc_sort_perm(int64_t n, const int32_t* key, const int32_t* id, int32_t* perm);

/* ---- simulation ---- */
orc_sim* orc_create(const orc_config* cfg);
void orc_destroy(orc_sim* s);
int orc_init(orc_sim* s, const orc_density* dens, const orc_laser* laser, int32_t fill);
int orc_step(orc_sim* s, int32_t nsteps);
/* Laser antenna on grid row `row` (1 .. nz-1): every later step adds the
 * current sheet J_y = -2 E_y'(t', z_a, x, y) / dz of `laser` after the filter.
 * NULL or row < 0 removes it.  -1 for a row out of range. */
int orc_set_antenna(orc_sim* s, const orc_laser* laser, int32_t row);
int orc_window_shift(orc_sim* s, int32_t ncells);
int orc_diagnostics(orc_sim* s, orc_diag* out, double* lineout /* nz or NULL */);
/* Threads (OpenMP) of the particle loop, whose per-thread current buffers
 * are summed after it, and of the laser initialisation, filter passes and
 * Yee updates, whose iterations write disjoint nodes; 1 by default.  Set
 * before orc_init for the laser.  -1 for n < 1, or n > 1 in a build without
 * OpenMP.  orc_max_threads: the OpenMP default thread count (1 without). */
int orc_set_threads(orc_sim* s, int32_t n);
int32_t orc_max_threads(void);

/* state access (domain rows i = 0..nz; layout [i][j][k], k = y fastest) */
int64_t orc_field_size(const orc_sim* s);
int orc_get_field(const orc_sim* s, int32_t comp, double* out);
int orc_set_field(orc_sim* s, int32_t comp, const double* in);
int64_t orc_num_pairs(const orc_sim* s);
/* arrays of length num_pairs; NULL pointers are skipped */
int orc_get_particles(const orc_sim* s, double* ze, double* xe, double* ye,
                      double* uz, double* ux, double* uy, double* zi, double* w,
                      int64_t* id);
int orc_add_pair(orc_sim* s, double ze, double xe, double ye, double uz, double ux,
                 double uy, double zi, double xi, double yi, double w, int64_t id);
void orc_clear_particles(orc_sim* s);
/* co-moving tile-major sort key of every live electron (see oracle source) */
int orc_sort_keys(const orc_sim* s, int32_t tz, int32_t tx, int32_t ty,
                  int64_t tz_min, int32_t ntz, int32_t* key, int32_t* id);
/* the laser vector potential and Ey' at one calculation-frame event (t', z', x, y) */
void orc_laser_eval(const orc_laser* L, int32_t dim, double gamma_b, double tp, double zp,
                    double x, double y, double* A, double* Ey);
/* the lab density profile set by orc_init at lab position z_lab, and the
 * channel factor at a transverse position (cells) */
double orc_lab_density(const orc_sim* s, double z_lab);
double orc_channel_factor(const orc_sim* s, double x, double y);
/* apply the configured current filter to one stored component in place */
int orc_filter_field(orc_sim* s, int32_t comp);

#ifdef __cplusplus
}
#endif
#endif
