/*
 * bfpic.h -- C ABI of the MI355X boosted-frame particle-in-cell library.
 *
 * One explicit electromagnetic PIC step in a Lorentz-boosted calculation frame
 * (Vay, Geddes, Cormier-Michel, Grote, "Effects of hyperbolic rotation in
 * Minkowski space on the modeling of plasma accelerators in a Lorentz boosted
 * frame"): field gather, relativistic Boris push, charge-conserving
 * (Esirkepov) current deposit, binomial current filter with compensation, Yee
 * FDTD update, with the boosted-frame laser and plasma initialisation, the
 * continuous plasma injection and the moving window around it.  The paper
 * motivates the frame (introduction; section "Effect of the hyperbolic
 * rotation") and the filtering (section "Mitigation of a numerical
 * instability") and defers the scheme itself to companion papers; the
 * textbook steps used are named at each entry point below.
 *
 * Units (normalised): time 1/omega0, length c/omega0 (lambda0 = 2 pi),
 * momentum u = gamma beta, E in m c omega0 / e, B in m omega0 / e, density in
 * n_crit.  Electrons carry q = -1, m = 1; each has a co-located ion partner of
 * opposite charge that moves rigidly with the lab-rest plasma.
 *
 * Conventions shared by every call
 *   - Every call returns a status: BFPIC_OK (0) or a negative BFPIC_ERR_*.
 *     On error nothing on the device has been modified and the message is
 *     available from bfpic_last_error().
 *   - All device memory is owned by the caller.  bfpic_query_sizes() reports
 *     one workspace size; the caller allocates that many bytes of device
 *     memory (256-byte aligned) and passes the pointer to bfpic_create().  The
 *     library keeps the pointer and never frees it; the workspace must outlive
 *     the context.
 *   - All device work is enqueued on the HIP stream given to bfpic_create()
 *     and is asynchronous unless a call says it synchronises.
 *   - One context per stream; a context is not thread-safe.
 *   - Field layout on the grid: component arrays indexed [i][j][k] with k (y)
 *     fastest, i over the z rows 0..nz, j over x, k over y (ny = 1 in 2D).
 *     Node (i, j, k) of a component sits at ((i+sz) dz, (j+sx) dx, (k+sy) dy)
 *     with the Yee offsets (sz, sx, sy): Ex (0,1/2,0), Ey (0,0,1/2),
 *     Ez (1/2,0,0), Bx (1/2,0,1/2), By (1/2,1/2,0), Bz (0,1/2,1/2); the y
 *     offsets are absent in 2D.
 */
#ifndef BFPIC_H
#define BFPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BFPIC_OK 0
#define BFPIC_ERR_ARG (-1)         /* bad argument, config or size */
#define BFPIC_ERR_CAPACITY (-2)    /* particle capacity too small */
#define BFPIC_ERR_HIP (-3)         /* a HIP runtime call failed */
#define BFPIC_ERR_STATE (-4)       /* call out of order (e.g. step before init) */
#define BFPIC_ERR_UNSUPPORTED (-5) /* option not implemented */

enum { BFPIC_FP64 = 0, BFPIC_FP32_SPLIT = 1 };
enum { BFPIC_BC_PERIODIC = 0, BFPIC_BC_MUR = 1 };
enum { BFPIC_LOAD_RANDOM = 0, BFPIC_LOAD_CENTERED = 1 };
enum { BFPIC_GATHER_MOMENTUM = 0, BFPIC_GATHER_ENERGY = 1 };

/* Field component ids for bfpic_get_field / bfpic_set_field. */
enum { BFPIC_EX = 0, BFPIC_EY, BFPIC_EZ, BFPIC_BX, BFPIC_BY, BFPIC_BZ,
       BFPIC_JX, BFPIC_JY, BFPIC_JZ };

typedef struct bfpic_config {
  int32_t dim;               /* 2: plane (z, x), y invariant; 3: (z, x, y) */
  int32_t nz, nx, ny;        /* cells per axis (ny ignored in 2D) */
  double dz, dx, dy;         /* cell sizes in the calculation frame */
  double cfl;                /* dt = cfl / sqrt(sum 1/d^2), 0 < cfl < 1 */
  int32_t shape_order;       /* 1 linear, 2 quadratic */
  int32_t filter_passes;     /* N binomial (1/4,1/2,1/4) passes per axis */
  int32_t filter_compensate; /* 1: one (-N/4, 1+N/2, -N/4) pass per axis */
  int32_t precision;         /* BFPIC_FP64 or BFPIC_FP32_SPLIT */
  int32_t deterministic;     /* 1: currents are summed as int64 fixed point
                                (unit 2^-e of the current, e fixed at init
                                from the largest particle weight), so results
                                do not depend on the order of atomic adds and
                                repeat bitwise from run to run */
  int32_t z_boundary;        /* BFPIC_BC_PERIODIC or BFPIC_BC_MUR */
  int32_t ppc;               /* macro-particles per lattice cell */
  int32_t load;              /* BFPIC_LOAD_RANDOM (SplitMix64) or _CENTERED */
  int32_t sort_interval;     /* steps between particle sorts; 0: never re-sort */
  uint64_t seed;             /* generator key of the in-cell positions */
  double beta_window;        /* window speed along +z (calculation frame) */
  int32_t auto_window;       /* 1: pic_step shifts the window on schedule */
  int32_t gather_form;       /* BFPIC_GATHER_MOMENTUM: every field component
                                interpolated with the deposit's shape on every
                                axis (momentum-conserving).  BFPIC_GATHER_ENERGY
                                (Galerkin, energy-conserving): along each axis
                                on which a component sits at half-integer nodes
                                it takes the shape of one order lower (nearest
                                half node for linear shapes, linear for
                                quadratic), the shape the charge-conserving
                                current of that component has along that axis.
                                One of the numerical levers against the
                                drifting-plasma instability (section
                                "Mitigation of a numerical instability": the
                                instability depends on the scheme's
                                smoothing and damping).  Witness electrons use
                                the same form. */
} bfpic_config;

/* Lab-frame plasma density.  nknots == 0: n_uniform everywhere.  nknots >= 2:
 * piecewise linear through (z_lab[m], n[m]) (host arrays, increasing z_lab),
 * zero outside.  du is a uniform momentum added to every electron at birth
 * (x, y, z order; zero for a cold plasma).  Plasma channel (the guiding
 * channel of the 10 GeV stage in the paper's last figure): the density is
 * multiplied by 1 + channel_depth r^2 / channel_radius^2, r the transverse
 * distance of the birth position from the laser axis (the box centre; x in
 * 2D, x and y in 3D).  channel_depth = 0: no channel; a Gaussian beam of
 * waist w0 is guided when the density rise at r = w0 is 4 / (k0 w0)^2 n_c.
 * ERR_ARG for channel_depth < 0, or > 0 with channel_radius <= 0. */
typedef struct bfpic_density {
  double n_uniform;
  int32_t nknots;
  const double* z_lab;
  const double* n;
  double du[3];
  double channel_depth;
  double channel_radius;
} bfpic_density;

/* Lab-frame laser: y-polarised paraxial Gaussian pulse along +z, given by its
 * vector potential A_y = a0 G(xi) Im[U(r, zeta) exp(i (xi + phase))],
 * xi = z - t - z_center, zeta = z - z_focus, G = exp(-xi^2/L^2) (cut at
 * |xi| > 4 L; L <= 0: no envelope), U the paraxial beam of 1/e waist w0
 * (w0 <= 0: plane; collimated = 1: exp(-r^2/w0^2) without diffraction).
 * The transverse axis is the box centre.  images_* > 0 sums that many
 * periodic images on each side (for periodic boxes). */
typedef struct bfpic_laser {
  double a0, w0, L, z_center, z_focus, phase;
  int32_t collimated;
  int32_t images_z, images_x, images_y;
} bfpic_laser;

/* Loss for the adjoint: L = (1 / nwin) sum over n = step_first .. step_last
 * of the mean of Ez^n over the node box i0..i1 (z rows of Ez, inclusive) by
 * j0..j1 (x columns, inclusive), where Ez^n is the field after step n (steps
 * counted from 1 after init) and nwin = step_last - step_first + 1; plus
 * witness_weight times the mean lab-frame energy gamma_b (gamma' + beta_b
 * u'_z) of the bound witness electrons after the last step (the
 * witness-beam energy; witness_weight = 0: no such term). */
typedef struct bfpic_loss {
  int32_t step_first, step_last;
  int32_t i0, i1, j0, j1;
  double witness_weight;
  int32_t k0, k1;  /* 3D: y nodes of the box; 2D: both 0 */
} bfpic_loss;

typedef struct bfpic_sizes {
  int64_t workspace_bytes;   /* total device bytes to allocate */
  int64_t field_bytes;       /* of which: fields */
  int64_t particle_bytes;    /* of which: particle arrays (both sort buffers) */
  int64_t scratch_bytes;     /* of which: tile, sort and diagnostic scratch */
} bfpic_sizes;

typedef struct bfpic_diag {
  int64_t step;
  double t;                  /* calculation-frame time */
  double window_cells;       /* total window displacement [cells] */
  double drift_cells;        /* D = step * beta_b dt / dz + window_cells */
  double ue, ub;             /* 1/2 sum E^2 dV, 1/2 sum B^2 dV over the domain */
  double ukin;               /* sum over electrons w (gamma - 1) */
  double ukin_drift;         /* sum over electrons w (gamma - gamma_b) */
  double wake_amp;           /* max |Ez| on the axis row */
  double gauss_res;          /* max |div E - F rho| over the checked nodes */
  double charge;             /* sum over electrons q w */
  int64_t live;              /* live electrons */
  int32_t nan_flag;          /* 1 if any field or particle value is not finite */
} bfpic_diag;

typedef struct bfpic_ctx bfpic_ctx;

/* ---- boost helper (host FP64, section "Effect of the hyperbolic rotation":
 *      the frame change is a rotation by rapidity artanh(beta_b)) ---- */
double bfpic_beta(double gamma);                 /* sqrt(gamma^2 - 1) / gamma */
double bfpic_drift_u(double gamma_b);            /* -gamma_b beta_b */
/* gamma_g = 1/sqrt(n_lab) (cold plasma, 1D) and the boosted group velocity
 * (beta_g - beta_b)/(1 - beta_g beta_b) without cancellation. */
double bfpic_group_gamma(double n_lab);
double bfpic_boosted_group_beta(double gamma_b, double n_lab);
/* Longitudinal resolution against the vacuum laser wavelength (section
 * "Mitigation of a numerical instability"): gamma_b (1 + beta_b) lambda0 / cells. */
double bfpic_boosted_dz(double gamma_b, double lambda0, double cells_per_wavelength);
double bfpic_yee_dt(int32_t dim, double dz, double dx, double dy, double cfl);

/* ---- lifecycle ---- */

/* Pure host.  Sizes of the device workspace for cfg and a particle capacity
 * (number of electrons; partners are implicit).  ERR_ARG on a bad config or
 * a capacity outside 1 .. 2^31 - 1 (the bound bfpic_create applies). */
int bfpic_query_sizes(const bfpic_config* cfg, int64_t particle_capacity, bfpic_sizes* out);

/* Creates a context on the current HIP device.  workspace: device pointer of
 * at least sizes.workspace_bytes, owned by the caller.  hip_stream: a
 * hipStream_t (NULL = the null stream).  ERR_ARG if the workspace is too small. */
int bfpic_create(const bfpic_config* cfg, int64_t particle_capacity, void* workspace,
                 int64_t workspace_bytes, void* hip_stream, bfpic_ctx** out);
void bfpic_destroy(bfpic_ctx* h);
const char* bfpic_last_error(const bfpic_ctx* h);

/* The boosted-frame initialisation.  The paper changes frame by a Lorentz
 * boost, which it describes as a hyperbolic rotation of space-time (section
 * "Effect of the hyperbolic rotation in Minkowski space"), and notes that
 * laser and plasma initialisation in the boosted frame need care (section
 * "Mitigation of a numerical instability"; the procedure itself is in its
 * companion papers).  This call sets the fields and particles at t' = 0 in
 * the frame boosted by gamma_boost along +z (gamma_boost = 1: lab frame).
 * Laser: the lab potential above is
 * evaluated on the t' = 0 hyperplane, i.e. at lab (t, z) = (gamma beta z',
 * gamma z'); Ey' = -dA/dt' there, B' = curl_h A' on the grid, and in 3D Ez'
 * from discrete div E' = 0 integrated from the low z end.  Plasma: every
 * lattice cell of the box gets ppc electrons with co-located ion partners,
 * u = (0, 0, -gamma_b beta_b) + du, weight gamma_b n_lab(z_lab) dV / ppc at
 * the lab birth coordinate z_lab = gamma_b z'.  n_e may be NULL (vacuum),
 * laser may be NULL (no laser).  Resets step, window and injection counters.
 * Particle ids: the lattice slot ((k ny + l) nx + j) ppc + s of column k,
 * transverse cell (j, l) and slot s, an int32; the columns a run may create
 * (the box plus every injected column) are bounded by
 * columns nx ny ppc <= 2^31.
 * ERR_ARG for more than 32 knots, knots that do not increase, a null knot
 * array or a bad channel; ERR_CAPACITY if the initial particles exceed the
 * capacity or the id space.  These checks run before anything is changed:
 * on them the context keeps its previous state.  A later failure (ERR_HIP)
 * leaves the context uninitialised. */
int init_boosted_plasma(bfpic_ctx* h, double gamma_boost, const bfpic_density* n_e,
                        const bfpic_laser* laser);

/* One explicit electromagnetic PIC step in the boosted frame, the step whose
 * cost the boosted frame reduces (introduction; section "Effect of the
 * hyperbolic rotation in Minkowski space": the speedup of the boosted-frame
 * run over the lab run), with the current filtering that keeps the
 * short-wavelength instability of the drifting plasma in check (section
 * "Mitigation of a numerical instability").  The steps are the textbook
 * methods: momentum-conserving gather with the deposit's shape, relativistic
 * Boris push (Boris 1970), Esirkepov's charge-conserving deposit (2001),
 * binomial filtering with compensation, Yee's FDTD update (1966) with
 * first-order Mur boundaries (1981).
 * Advances nsteps full steps.  Each step: inject the lattice columns whose low
 * edge has entered the box (k - D < nz), re-sort the particles if the sort
 * interval is due, then gather -> Boris (split drift form) -> move ->
 * Esirkepov deposit of each electron and its drifting partner -> filter J ->
 * B half step, E full step (+ Mur), B half step; then drop pairs more than
 * order+1 cells outside [0, nz] along z.  With auto_window the window shifts
 * after a step by floor(beta_window t / dz) - window_cells.  Asynchronous.
 * ERR_CAPACITY (before that step's launches) if its injections would not fit
 * the capacity or the id space; the steps before it have run. */
int pic_step(bfpic_ctx* h, int32_t nsteps);

/* The moving window that follows the laser (section "Effect of the
 * hyperbolic rotation in Minkowski space": the lab-frame simulation window
 * moves with the laser; in the boosted frame it moves at the boosted group
 * velocity, and near the laser's frame it stands still).
 * Shifts the window by ncells (either sign): field rows move by ncells,
 * the rows that enter are zero, particles keep their lab positions (their
 * grid coordinates drop by ncells).  Columns that become due are injected by
 * the next pic_step.  ERR_ARG on a periodic z boundary.  Asynchronous. */
int moving_window_shift(bfpic_ctx* h, int32_t ncells);

/* Host FP64 schedule: floor(beta_window t / dz) - window_cells. */
int bfpic_window_due(bfpic_ctx* h, int32_t* ncells);

/* Diagnostics of the run: the field and kinetic energies and the on-axis
 * wake field Ez whose amplitude sets a stage's energy gain (section
 * "Modeling of up to 1 TeV stages", Fig. 4), and the Gauss-law residual and
 * non-finite flag that show a run is sound.  U_E = 1/2 sum E^2 dV,
 * U_B = 1/2 sum B^2 dV over the domain nodes of each component,
 * U_kin = sum w (gamma - 1) over electrons; all sums in FP64.
 * Fills *out (host) with FP64 diagnostics.  lineout_dev (may be NULL): device
 * buffer of nz doubles that receives Ez on the axis row (j = nx/2, k = ny/2).
 * mask is reserved (pass 0xffffffff).  Synchronises the stream. */
int diagnostics(bfpic_ctx* h, uint32_t mask, bfpic_diag* out, double* lineout_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * diagnostics as diagnostics(), with the same arguments and results, whose
 * reduction scratch (block partials, final values, non-finite flag) lives
 * in a static device array of 32 KiB that the library holds on each device
 * until the process ends, instead of the context's workspace.  The charge
 * grids of the Gauss residual are the context's own, inside the workspace
 * the caller passed to bfpic_create.  The call allocates nothing and clears
 * what it reads with fill kernels (no memset).  Every call on one device
 * shares that array: calls that overlap on one device (contexts on
 * different streams, or different threads) race and must be serialised by
 * the caller.  ERR_STATE if the context's device is not current or before
 * init; ERR_HIP if the array's device address cannot be resolved;
 * ERR_ARG if the reductions would need more than the array holds (they are
 * capped below it).  Synchronises the stream. */
int diagnostics_noalloc(bfpic_ctx* h, uint32_t mask, bfpic_diag* out, double* lineout_dev);

/* ---- lab-frame and spectral diagnostics of the on-axis laser field ---- */

/* Where and when a record was taken: boosted-frame time t' = step dt, the
 * boosted position of row 0 z0' = window_cells dz (row i lies at
 * z0' + i dz'), the row spacing, the number of rows n = nz + 1 and the boost. */
typedef struct bfpic_axis_meta {
  int64_t step;
  double t_prime, z0_prime, dz_prime;
  int32_t n;
  double gamma_b, beta_b;
} bfpic_axis_meta;

/* On-axis history of the transverse laser field, the quantity whose
 * boosted-frame and Lorentz-transformed histories are compared in the
 * section "Effect of the hyperbolic rotation in Minkowski space" (Fig. 2).
 * Writes rows i = 0..nz of the axis row (j = nx/2, k = ny/2) into out_dev
 * (device, nz + 1 doubles):
 *   frame 0: the boosted-frame E'_y at its nodes;
 *   frame 1: the lab-frame field at the same events, E_y = gamma_b (E'_y -
 *            beta_b B'_x) (inverse transform of the transverse fields, c = 1),
 *            with B'_x, stored at half rows, averaged onto row i.
 * Fields at integer time (after the last completed step).  *meta (host, may
 * be NULL) receives the record's place and time.  ERR_ARG for a frame other
 * than 0 or 1 or a NULL out_dev, ERR_STATE before init.  Asynchronous. */
int bfpic_axis_record(bfpic_ctx* h, int32_t frame, double* out_dev, bfpic_axis_meta* meta);

/* Lorentz transform of a record history to the lab frame (section "Effect of
 * the hyperbolic rotation in Minkowski space": boosted data shown in the
 * laboratory-frame moving window).  rec_dev: nrec records of n doubles
 * (record r, row i at rec_dev[r n + i]); t_prime_dev, z0_prime_dev: per
 * record t' (strictly increasing) and z0' (device arrays of nrec doubles);
 * dz_prime: row spacing.  Output (device, nt x nzeta doubles, row-major in
 * t): the value at lab time t_m = t0 + m dt and window coordinate
 * zeta_k = zeta0 + k dzeta, i.e. at z = zeta_k + v_window t_m, read at the
 * boosted event t' = gamma_b (t - beta_b z), z' = gamma_b (z - beta_b t) by
 * linear interpolation along z' within the two records that bracket t', then
 * linearly in t'; NaN where that event lies outside the recorded rows or
 * times.  FP64.  ERR_ARG for nrec < 2, n < 2, nt < 1, nzeta < 1,
 * dz_prime <= 0, gamma_b < 1 or a NULL pointer.  Asynchronous. */
int bfpic_back_transform(bfpic_ctx* h, const double* rec_dev, const double* t_prime_dev,
                         const double* z0_prime_dev, int64_t nrec, int32_t n,
                         double dz_prime, double gamma_b, double t0, double dt, int32_t nt,
                         double zeta0, double dzeta, int32_t nzeta, double v_window,
                         double* out_dev);

/* Spectral content of each record, as in the spectral content histories of
 * the section "Mitigation of a numerical instability" (Fig. 3): the power
 * |X_q|^2 of the discrete Fourier transform X_q = sum_i x_i exp(-2 pi i q i / m)
 * of record r zero-padded to m points, for q = 0..m/2 (wavenumber
 * 2 pi q / (m dz')), into out_dev[r (m/2 + 1) + q].  rec_dev as for
 * bfpic_back_transform; m a power of two, 2 <= m <= 8192, 1 <= n <= m (longer
 * records: pass a window of them).  FP64, radix-2 in LDS.  ERR_ARG
 * otherwise.  Asynchronous. */
int bfpic_axis_spectrum(bfpic_ctx* h, const double* rec_dev, int64_t nrec, int32_t n, int32_t m,
                        double* out_dev);

/* ---- witness electrons (section "Modeling of up to 1 TeV stages", Fig. 4:
 * energy gain of the accelerated beam against laboratory position) ---- */

/* Binds n witness electrons: test particles that feel the run's fields and
 * deposit no current.  state_dev: caller-owned device array of n rows of six
 * FP64 values (z, x, y, u_z, u_x, u_y), position in grid cells relative to
 * the window, momentum of the calculation frame; it must stay valid while
 * bound.  Each pic_step then, before the plasma moves, gathers E and B at
 * every witness from the start-of-step fields with the deposit's shape (the
 * working-precision grid read as FP64; no field beyond rows 0..nz in open
 * z), applies the relativistic Boris rotation in FP64 with charge -1 and
 * moves it by v dt (x, y periodic; z wraps in a periodic box); a window
 * shift lowers every z by the shift.  Witnesses leave no mark on the
 * fields or the plasma.  n = 0 unbinds; init_boosted_plasma unbinds.  A
 * taped adjoint run carries the bound witnesses (bind them before sizing
 * its tape), and its loss may weigh their final lab energy.
 * ERR_ARG for n < 0 or a null array with n > 0, ERR_STATE before init.
 * Calls on one context are ordered on its stream. */
int bfpic_witness_bind(bfpic_ctx* h, int32_t n, double* state_dev);

/* Laboratory view of the bound witnesses into out_dev (n rows of four FP64
 * values): lab time, lab position, gamma and u_z of the event (t', z') with
 * t' = step dt, z' = (z + window cells) dz, the momentum boosted back from
 * the frame moving at +beta_b along z: t = gamma_b (t' + beta_b z'),
 * z = gamma_b (z' + beta_b t'), gamma = gamma_b (gamma' + beta_b u'_z),
 * u_z = gamma_b (u'_z + beta_b gamma').  ERR_STATE with none bound.
 * Asynchronous. */
int bfpic_witness_lab(bfpic_ctx* h, double* out_dev);

/* ---- checkpoint and resume ---- */

/* Device bytes of a state blob of the present state (call right before
 * pic_save: the size follows the number of particle slots in use).
 * ERR_STATE before init. */
int bfpic_state_bytes(bfpic_ctx* h, int64_t* bytes);

/* Writes the simulation state into blob_dev, a caller-owned device buffer of
 * at least bfpic_state_bytes bytes, 256-byte aligned: a header (the
 * configuration, the step and window schedule, the injection cursor, the
 * boost and density parameters, the fixed-point scale), then E and B with
 * their guard rows, the particle slots in use and the device counters.
 * Currents and scratch are rebuilt within each step and are not saved, nor
 * are bound witnesses (caller state).  The blob may be copied to the host
 * and back unchanged.  ERR_ARG for a short or misaligned blob, ERR_STATE
 * before init.  Synchronises. */
int pic_save(bfpic_ctx* h, void* blob_dev, int64_t blob_bytes);

/* Restores a state written by pic_save into a context created with the same
 * configuration (grid, spacings, CFL, shapes, filter, precision,
 * deterministic mode, boundaries, loading, seed and window; capacity and
 * sort interval may differ), then re-sorts the particles into tiles.  The
 * run continues from the saved step; in deterministic mode it continues
 * bitwise as the uninterrupted run would.  ERR_ARG for a blob that is not a
 * state, comes from another configuration or is shorter than its header
 * says, ERR_CAPACITY if its slots exceed the capacity; these leave the
 * context untouched.  After ERR_HIP the context's state is undefined
 * (re-initialise or load again).  Synchronises. */
int pic_load(bfpic_ctx* h, const void* blob_dev, int64_t blob_bytes);

/* Laser antenna (an alternative to placing the laser in the box at init;
 * the paper's boosted runs start with the laser in the box, section "Effect
 * of the hyperbolic rotation", so the antenna extends the method rather than
 * following a passage of it): from the next pic_step on, every step adds to the filtered current on grid
 * row `row` (1 .. nz-1) the sheet J_y = -2 E_y'(t', z_a, x, y) / dz, which
 * radiates the boosted field E_y' of `laser` (as init_boosted_plasma would
 * place it, same parameters and images) into both directions: a surface
 * current K radiates E_y = -K/2 on either side in 1D vacuum.  t' is the step's
 * mid time and z_a = (row + window cells) dz (the row moves with the window).
 * The source is not filtered.  laser = NULL removes the antenna;
 * init_boosted_plasma removes it too, and pic_save does not record it.
 * ERR_STATE before init, ERR_ARG for a row out of range or bad laser
 * parameters.  A taped adjoint run refuses a context with an antenna
 * (ERR_UNSUPPORTED). */
int bfpic_antenna(bfpic_ctx* h, const bfpic_laser* laser, int32_t row);

/* ---- state access (tests and tools; asynchronous unless stated) ---- */

/* Copies component comp at integer time (domain rows 0..nz; row nz is zero
 * where the component has no node there) into out_dev, FP64, shape
 * (nz+1) x nx x ny.  For J the last step's filtered current. */
int bfpic_get_field(bfpic_ctx* h, int32_t comp, double* out_dev);
/* Overwrites E or B component comp from in_dev (same layout). */
int bfpic_set_field(bfpic_ctx* h, int32_t comp, const double* in_dev);

/* Number of particle slots in use (live + not yet compacted).  Synchronises. */
int bfpic_num_slots(bfpic_ctx* h, int64_t* n);

/* Exports every slot as absolute FP64 state into device arrays of at least
 * bfpic_num_slots entries: electron position z, x, y (grid cells, relative to
 * the window), momentum (ux, uy, uz), weight, id (-1: removed). */
int bfpic_get_particles(bfpic_ctx* h, double* z, double* x, double* y, double* ux,
                        double* uy, double* uz, double* w, int32_t* id);

/* Forces a particle sort now: co-moving tile-major cell keys, ties by id;
 * then, inside each tile of at most 512 cells, particles are ordered by their
 * rank within their cell and then by cell, so that consecutive particles lie
 * in distinct cells. */
int bfpic_sort(bfpic_ctx* h);

/* The last sort: the key and id of every source slot, and perm[d] = source
 * slot of destination d (live particles only, in the order bfpic_sort
 * describes).  Device arrays of at least
 * bfpic_num_slots entries before that sort.  *n (host) receives the number of
 * source slots and *n_live the number of sorted live particles; *tz_min,
 * *ntz (host) the co-moving tile rows used for the keys.  Synchronises. */
int bfpic_last_sort(bfpic_ctx* h, int32_t* key_dev, int32_t* id_dev, int32_t* perm_dev,
                    int64_t* n, int64_t* n_live, int64_t* tz_min, int32_t* ntz);

/* The sort probe: perm[d] = source slot of destination d of the last sort
 * (the permutation bfpic_last_sort also returns), for live particles only;
 * *n_live (host) receives their number.  perm_dev: device array of at least
 * bfpic_num_slots entries before that sort.  ERR_STATE before any sort.
 * Synchronises. */
int bfpic_sort_permutation(bfpic_ctx* h, int32_t* perm_dev, int64_t* n_live);

/* Tile geometry used by the sort key: tile sizes along z, x, y in cells. */
int bfpic_tile_shape(const bfpic_ctx* h, int32_t* tz, int32_t* tx, int32_t* ty);

/* Per-kernel timing with HIP events on the context's stream.  enable = 1
 * starts recording (and clears totals).  bfpic_kernel_time synchronises and
 * returns the summed milliseconds and launch count of a kernel class:
 * 0 gather-push-deposit (tiled), 1 the same on the global path (unsorted tail
 * and stragglers), 2 current fold + filter, 3 Yee (both half steps, E, Mur),
 * 4 sort, 5 injection, 6 window shift. */
int bfpic_kernel_timing(bfpic_ctx* h, int32_t enable);
int bfpic_kernel_time(bfpic_ctx* h, int32_t cls, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------------------
 * Adjoint (2D and 3D).  The paper prints no adjoint; these calls give the exact
 * discrete gradient of a field loss (bfpic_loss) through the step above with
 * respect to the laser amplitude a0 and the lab density profile (the knot
 * values of init_boosted_plasma, or n_uniform), the two inputs that set a
 * stage's wake.  The reverse sweep runs the transposes of the Yee update, the
 * Mur boundary and the filter, and per particle the vector-Jacobian product of
 * gather, push, move and deposit, backwards over the steps, recomputing each
 * segment of `interval` steps from its checkpoint.  Bound witness electrons
 * are carried: their states are taped, and with a witness term in the loss
 * their vector-Jacobian product (gather, push, move) is run backwards too,
 * its gathered-field part added to the field adjoint.  With auto_window the
 * taped run shifts the window as pic_step does (the loss reads each step's
 * shifted state) and the reverse sweep applies the shift's transpose;
 * particles are not re-sorted during a taped run.
 *
 * bfpic_adjoint_tape_bytes: device bytes of the tape for nsteps steps with a
 *   checkpoint every `interval` steps (checkpoints, one segment of per-step
 *   state, adjoint arrays).  The caller allocates it (256-byte aligned).
 * bfpic_forward_loss: from the state right after init_boosted_plasma, runs
 *   nsteps steps, storing the checkpoints in `tape`, and returns the loss in
 *   *loss_out (host).  The tape must stay allocated for pic_step_adjoint.
 *   Synchronises.  ERR_STATE if steps were taken since init.
 * pic_step_adjoint: reverse sweep of the last bfpic_forward_loss run:
 *   *dL_da0 (host) and dL_dn[m] (host array of nn >= number of knots, or >= 1
 *   for a uniform density).  Leaves the simulation state unspecified
 *   (re-initialise before stepping on), witness states included.
 *   ERR_STATE if the bound witnesses changed since the taped run.
 *   Synchronises. */
int bfpic_adjoint_tape_bytes(bfpic_ctx* h, int32_t nsteps, int32_t interval, int64_t* bytes);
int bfpic_forward_loss(bfpic_ctx* h, int32_t nsteps, int32_t interval, const bfpic_loss* loss,
                       void* tape, int64_t tape_bytes, double* loss_out);
int pic_step_adjoint(bfpic_ctx* h, double* dL_da0, double* dL_dn, int32_t nn);
/* The per-particle vector-Jacobian product of pic_step_adjoint is formed by
 * stages by default (gather, push and deposit each evaluated once with one
 * tangent per input of the stage).  enable != 0 selects instead one dual
 * evaluation of the whole particle step per input direction (twelve): the
 * same product by another route, kept as a reference for tests.  Takes
 * effect at the next pic_step_adjoint.  ERR_ARG for a null context. */
int bfpic_adjoint_per_direction(bfpic_ctx* h, int32_t enable);

#ifdef __cplusplus
}
#endif
#endif
