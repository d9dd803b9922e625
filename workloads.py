"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

Plain numbers only: each workload states its grid, frame, plasma, laser and
numerics in the paper's terms (cells per boosted laser wavelength, lengths in
vacuum laser wavelengths lambda0, lab densities in n_crit).  Turning them into
cell sizes, time steps, window speeds and lab-frame laser positions is done by
``resolve_gpu`` with the HIP library's own boost helper and by
``resolve_oracle`` with the oracle's own helper; the two never share a helper.

The paper measures on physical stages (densities 1e19..1e15 cm^-3, the caption
of Fig. 4) whose parameters are in companion papers; these synthetic
configurations stand in for them.  Random numbers are drawn by each side from
the same counter-based generator (SplitMix64) keyed by ``seed``.
"""
import math

LAMBDA0 = 2.0 * math.pi  # vacuum laser wavelength in units of c / omega0

# --------------------------------------------------------------------------
# lab_2d:       plain lab-frame 2D3V run (FP64), periodic box, 200 steps
# boost13_2d:   gamma_boost = 13, 2048 x 256, moving window, FP32 split
# boost130_2d:  gamma_boost = 130, 8192 x 512, FP32 split (throughput headline)
# boost100_3d:  gamma_boost = 100, 3D3V quadratic, 512 x 128 x 128, FP32 split
# The *_small variants keep the physics of their parent (frame, resolution rule,
# density, laser, numerics) on a grid the oracle finishes in seconds.
# --------------------------------------------------------------------------
WORKLOADS = {
    "lab_2d": dict(
        dim=2, nz=128, nx=64, ny=1, gamma_b=1.0, dz_lambda0=1 / 16, dx_lambda0=1 / 16,
        cfl=0.95, n_lab=0.01, ppc=4, order=1, filter_passes=1, filter_compensate=0,
        zbc="periodic", precision="fp64", steps=200, seed=1012, window=None,
        laser=dict(a0=1.0, w0_lambda0=8.0, L_lambda0=4.0, place="box_center", collimated=1,
                   images_z=3, images_x=12)),
    "boost13_2d": dict(
        dim=2, nz=2048, nx=256, ny=1, gamma_b=13.0, dz_cells_per_wavelength=16, dx_lambda0=0.25,
        cfl=0.95, n_lab=1e-3, ppc=8, order=1, filter_passes=4, filter_compensate=1, zbc="mur",
        precision="fp32", steps=2000, seed=1013, window="group",
        laser=dict(a0=1.0, w0_lambda0=8.0, L_lambda0=4.0, place="front", front_gap=4.5,
                   collimated=1)),
    "boost130_2d": dict(
        dim=2, nz=8192, nx=512, ny=1, gamma_b=130.0, dz_cells_per_wavelength=16,
        dx_lambda0=0.5, cfl=0.95, n_lab=1e-4, ppc=8, order=1, filter_passes=4,
        filter_compensate=1, zbc="mur", precision="fp32", steps=5000, seed=1014, window=None,
        laser=dict(a0=1.0, w0_lambda0=8.0, L_lambda0=4.0, place="front", front_gap=4.5,
                   collimated=1)),
    "boost100_3d": dict(
        dim=3, nz=512, nx=128, ny=128, gamma_b=100.0, dz_cells_per_wavelength=16,
        dx_lambda0=0.5, dy_lambda0=0.5, cfl=0.95, n_lab=3e-4, ppc=2, order=2, filter_passes=4,
        filter_compensate=1, zbc="mur", precision="fp32", steps=1000, seed=1015, window="group",
        laser=dict(a0=2.0, w0_lambda0=10.0, L_lambda0=4.0, place="front", front_gap=4.5,
                   collimated=1)),
}


# adjoint_2d: gamma_boost = 13, 1024 x 128, 4 ppc, 500 steps, a checkpoint every
# 50 steps; lab density 1e-3 n_crit times a 16-knot piecewise-linear profile
# (values 1 +- 0.1, seeded) over the lab length that crosses the box; loss =
# mean of Ez over the last 100 steps in a box behind the pulse on axis.
WORKLOADS["adjoint_2d"] = dict(
    dim=2, nz=1024, nx=128, ny=1, gamma_b=13.0, dz_cells_per_wavelength=16, dx_lambda0=0.5,
    cfl=0.95, n_lab=1e-3, ppc=4, order=1, filter_passes=4, filter_compensate=1, zbc="mur",
    precision="fp32", steps=500, seed=1016, window=None, interval=50, nknots=16,
    loss_steps=100,
    laser=dict(a0=1.0, w0_lambda0=8.0, L_lambda0=4.0, place="front", front_gap=4.5,
               collimated=1))


def adjoint_setup(W, dz, beta, dt, beta_window=0.0):
    """Density knots (lab z, values), loss window and Ez box of an adjoint run.

    The knots cover the lab length of every lattice column the run holds
    (the box at t' = 0 plus the columns injected over the run, as the plasma
    drifts in and, with a moving window at beta_window, as the window
    advances).  The box spans
    rows [i_L - 2.5 L', i_L - L'] behind the pulse centre i_L (L' the boosted
    envelope length in cells), |j - nx/2| <= 4: within the 500 steps of the
    adjoint configuration the wake forms just behind the pulse (an FP64 run
    puts its on-axis Ez, ~1e-3, at rows 576..671 over steps 400..500, with
    the pulse centre at row 736 at t' = 0); a box too short for that (a pulse
    as long as a small box) is 9 rows centred on i_L."""
    import numpy as np
    g = W["gamma_b"]
    sb = (beta(g) + abs(beta_window)) * dt / dz
    cols = W["nz"] + W["steps"] * sb + 8
    nk = W.get("nknots", 4)
    kz = list(np.linspace(-2.0 * g * dz, g * dz * cols, nk))
    rng = np.random.default_rng(W["seed"])
    kn = list(W["n_lab"] * (1.0 + 0.1 * rng.uniform(-1.0, 1.0, nk)))
    las = W["laser"]
    doppler = 1.0 / (g * (1.0 + beta(g)))
    L = las["L_lambda0"] * LAMBDA0
    if las["place"] == "box_center":
        iL = 0.5 * W["nz"]
    else:
        iL = W["nz"] - las["front_gap"] * L / doppler / dz
    Lc = L / doppler / dz
    i0 = int(max(0, np.floor(iL - 2.5 * Lc)))
    i1 = int(min(W["nz"] - 1, np.ceil(iL - Lc)))
    if i1 - i0 < 8:  # a box shorter than that: 9 rows centred on iL
        i0, i1 = int(max(0, iL - 4)), int(min(W["nz"] - 1, iL + 4))
    j0, j1 = W["nx"] // 2 - 4, W["nx"] // 2 + 4
    box = (i0, i1, j0, j1)
    if W["dim"] == 3:  # the same extent along y
        box += (W["ny"] // 2 - 4, W["ny"] // 2 + 4)
    n = W["steps"]
    win = (n - W.get("loss_steps", max(1, n // 5)) + 1, n)
    return dict(knots_z=kz, knots_n=kn, box=box, window=win,
                interval=W.get("interval", 10))


def small(name, **over):
    """A smaller box with the physics of `name`; the pulse sits at the box centre."""
    w = dict(WORKLOADS[name])
    w["laser"] = dict(w["laser"], place="box_center")
    w.update(over)
    return w


WORKLOADS["boost13_2d_small"] = small("boost13_2d", nz=256, nx=64, ppc=4, steps=100)
WORKLOADS["boost130_2d_small"] = small("boost130_2d", nz=256, nx=64, ppc=4, steps=100)
WORKLOADS["boost100_3d_small"] = small("boost100_3d", nz=48, nx=16, ny=16, steps=30)
# wide enough in x and y (24 >= the 17-node region of a quadratic 8^3 tile) to
# run the tiled 3D path
WORKLOADS["boost100_3d_tiled"] = small("boost100_3d", nz=48, nx=24, ny=24, steps=20)
WORKLOADS["lab_2d_fp32"] = small("lab_2d", precision="fp32")
SMOKE = small("boost13_2d", nz=96, nx=64, ppc=2, steps=20, precision="fp64")
WORKLOADS["adjoint_2d_small"] = small("adjoint_2d", nz=128, nx=32, ppc=2, steps=60,
                                      interval=10, nknots=5, loss_steps=20)
WORKLOADS["adjoint_2d_tiny"] = small("adjoint_2d", nz=64, nx=16, ppc=2, steps=40,
                                     interval=10, nknots=4, loss_steps=10)
# the adjoint's 3D case: the same physics in a 32 x 16 x 16 box (dy = dx),
# 1 pair per cell, 24 steps, a checkpoint every 8
WORKLOADS["adjoint_3d_tiny"] = small("adjoint_2d", dim=3, nz=32, nx=16, ny=16, dy_lambda0=0.5,
                                     ppc=1, steps=24, interval=8, nknots=4, loss_steps=8)
# Drifting cold plasma without laser, periodic z: the high-frequency numerical
# instability of a plasma streaming through the grid at -beta_b, and its
# mitigation by filtering the current.  An undisturbed pair deposits nothing,
# so the plasma is seeded with a uniform transverse birth momentum
# (INSTABILITY_SEED_DU); the random in-cell positions make the seed noisy.
INSTABILITY_SEED_DU = (1.0e-3, 0.0, 0.0)
WORKLOADS["drift_instability_2d"] = small("boost130_2d", nz=256, nx=64, ppc=4, steps=2000,
                                          zbc="periodic", window=None)
WORKLOADS["drift_instability_2d_small"] = small("boost130_2d", nz=128, nx=32, ppc=2, steps=600,
                                                zbc="periodic", window=None, precision="fp64")

# On-axis laser history in vacuum at gamma_boost = 5 (one of the boosts of the
# hyperbolic-rotation comparison), FP64, no window: the boosted-frame record
# history and its Lorentz transform to the lab frame.  The pulse is uniform
# across the periodic box (waist 1e4 lambda0), so that it propagates as the
# 1D pulse its analytic lab field describes.
WORKLOADS["lab_history_2d"] = small(
    "boost13_2d", gamma_b=5.0, nz=256, nx=32, ppc=1, steps=60, window=None, precision="fp64",
    laser=dict(WORKLOADS["boost13_2d"]["laser"], place="box_center", w0_lambda0=1.0e4))


def _resolve(W, beta, boosted_dz, yee_dt, group_beta):
    g = W["gamma_b"]
    if "dz_cells_per_wavelength" in W:
        dz = boosted_dz(g, LAMBDA0, W["dz_cells_per_wavelength"])
    else:
        dz = W["dz_lambda0"] * LAMBDA0
    dx = W["dx_lambda0"] * LAMBDA0
    dy = W.get("dy_lambda0", 1.0 / LAMBDA0) * LAMBDA0
    dt = yee_dt(W["dim"], dz, dx, dy, W["cfl"])
    bw = group_beta(g, W["n_lab"]) if W.get("window") == "group" else 0.0
    las = W["laser"]
    b = beta(g)
    doppler = 1.0 / (g * (1.0 + b))  # gamma (1 - beta): lab -> frame wavenumber factor
    L = las["L_lambda0"] * LAMBDA0
    if las["place"] == "box_center":
        zc_frame = 0.5 * W["nz"] * dz
    else:  # centre front_gap envelope lengths behind the front edge of the box
        zc_frame = W["nz"] * dz - las["front_gap"] * L / doppler
    laser = dict(a0=las["a0"], w0=las["w0_lambda0"] * LAMBDA0, L=L,
                 z_center=doppler * zc_frame, z_focus=g * zc_frame, phase=0.0,
                 collimated=las.get("collimated", 0), images_z=las.get("images_z", 0),
                 images_x=las.get("images_x", 0), images_y=las.get("images_y", 0))
    return dict(dz=dz, dx=dx, dy=dy, dt=dt, beta_window=bw, laser=laser)


def resolve_gpu(W, precision=None, sort_interval=20, capacity=None):
    """HIP library config, init arguments and step count of a workload."""
    import paper_1011_0917_amd as P
    r = _resolve(W, P.beta, P.boosted_dz, P.yee_dt, P.boosted_group_beta)
    prec = precision or W["precision"]
    cfg = P.make_config(
        dim=W["dim"], nz=W["nz"], nx=W["nx"], ny=W.get("ny", 1), dz=r["dz"], dx=r["dx"],
        dy=r["dy"], cfl=W["cfl"], shape_order=W["order"], filter_passes=W["filter_passes"],
        filter_compensate=W["filter_compensate"],
        precision=P.FP64 if prec == "fp64" else P.FP32_SPLIT,
        z_boundary=P.BC_PERIODIC if W["zbc"] == "periodic" else P.BC_MUR, ppc=W["ppc"],
        load=W.get("load", 0), sort_interval=sort_interval, seed=W["seed"],
        beta_window=r["beta_window"], auto_window=1 if W.get("window") else 0,
        gather_form=P.GATHER_ENERGY if W.get("gather") == "energy" else P.GATHER_MOMENTUM)
    cells = W["nz"] * W["nx"] * W.get("ny", 1)
    if capacity is None:
        # initial plasma + injected columns over the run + margin
        capacity = int(cells * W["ppc"] * 1.15) + 64 * W["nx"] * W.get("ny", 1) * W["ppc"]
    init = dict(gamma_b=W["gamma_b"], n_lab=W["n_lab"], laser=P.make_laser(**r["laser"]),
                capacity=capacity)
    return cfg, init, W["steps"]


def resolve_oracle(W):
    """Oracle Sim keyword arguments and init arguments of a workload."""
    import oracle as O

    def group_beta(g, n):
        return O.boosted_group_beta(g, n)

    r = _resolve(W, O.beta_of_gamma, O.boosted_dz, O.yee_dt, group_beta)
    kw = dict(dim=W["dim"], nz=W["nz"], nx=W["nx"], ny=W.get("ny", 1), dz=r["dz"], dx=r["dx"],
              dy=r["dy"], dt=r["dt"], order=W["order"], filter_passes=W["filter_passes"],
              filter_compensate=W["filter_compensate"],
              zbc=0 if W["zbc"] == "periodic" else 1, ppc=W["ppc"], seed=W["seed"],
              gamma_b=W["gamma_b"], beta_window=r["beta_window"],
              auto_window=1 if W.get("window") else 0, ions=1, load=W.get("load", 0),
              gather=1 if W.get("gather") == "energy" else 0)
    init = dict(n_lab=W["n_lab"], laser=O.make_laser(**r["laser"]))
    return kw, init


# Witness beam: n test electrons in the wake behind the laser (the accelerated
# beam whose energy gain against lab position is tracked), seeded: z uniform
# over [0.15, 0.40] of the box, x (and y) uniform within nx/8 (ny/8) of the
# axis, calculation-frame momentum u'_z uniform in [0.5, 3.0] and transverse
# momenta normal with standard deviation 0.02.  Rows (z, x, y, u_z, u_x, u_y).
def witness_beam(W, n, seed=None):
    import numpy as np
    rng = np.random.default_rng(W["seed"] + 7 if seed is None else seed)
    nz, nx, ny = W["nz"], W["nx"], W.get("ny", 1)
    out = np.zeros((n, 6))
    out[:, 0] = rng.uniform(0.15 * nz, 0.40 * nz, n)
    out[:, 1] = nx / 2 + rng.uniform(-nx / 8, nx / 8, n)
    if W["dim"] == 3:
        out[:, 2] = ny / 2 + rng.uniform(-ny / 8, ny / 8, n)
    out[:, 3] = rng.uniform(0.5, 3.0, n)
    out[:, 4] = rng.normal(0.0, 0.02, n)
    out[:, 5] = rng.normal(0.0, 0.02, n)
    return out


# Energy-gain scaling of the accelerated beam (the rescaled gain-versus-lab-
# position curves of Fig. 4), downscaled to four lab densities n = 2e-3, 1e-3,
# 5e-4, 2.5e-4 n_c, each in the frame gamma_b = gamma_g / 2 (gamma_g = n^-1/2):
#   (gamma_b = ratio gamma_g for the frame comparison)
#   * a resonant plane-wave pulse: a0 = 1, Gaussian length L = sqrt(2) / k_p,
#     uniform across a periodic slab of 16 transverse cells (no diffraction,
#     as no guiding channel is modelled), its centre 4.5 boosted lengths
#     (72 L / lambda0 cells) behind the front of the box;
#   * 16 cells per boosted laser wavelength along z, transverse cells of
#     16 lambda0 and Courant number 0.99 (c dt / dz' = 0.96 to 0.99), 4 pairs
#     per cell, FP32 split, window at the boosted group velocity;
#   * current filter: 8 binomial passes with compensation up to gamma_b = 16,
#     16 passes above (wider filtering at the higher boosts);
#   * box: the pulse's front gap plus 2.5 boosted wake periods (wake_cells);
#     run: 2.4 dephasing lengths lambda_p^3 / lambda0^2 of lab travel;
#   * witnesses: 256 on axis, evenly over 1.5 wake periods behind the pulse,
#     at lab gamma 2 gamma_g.
# The same stage at 1e-3 n_c is also run in the frame gamma_b = 0.85 gamma_g
# (box and run length by the same rules), for the lab energy gain's
# independence of the calculation frame.
GAIN_DENSITIES = (2e-3, 1e-3, 5e-4, 2.5e-4)
_GAIN_BOX = {(2e-3, 0.5): (1280, 1100, 286.5), (1e-3, 0.5): (1536, 1550, 405.0),
             (5e-4, 0.5): (2304, 2210, 572.6), (2.5e-4, 0.5): (3072, 3160, 809.7),
             (1e-3, 0.85): (1280, 750, 293.8)}  # nz, steps, wake_cells


def gain_scaling(n, ratio=0.5):
    nz, steps, wake = _GAIN_BOX[(n, ratio)]
    kp = math.sqrt(n)
    L_l0 = math.sqrt(2.0) / kp / LAMBDA0
    gb = ratio / kp
    W = small("boost13_2d", nz=nz, nx=16, ppc=4, gamma_b=gb, n_lab=n, dx_lambda0=16.0,
              cfl=0.99, filter_passes=8 if gb <= 16.0 else 16, precision="fp32",
              window="group", steps=steps,
              laser=dict(a0=1.0, w0_lambda0=1.0e4, L_lambda0=L_l0, place="front",
                         front_gap=4.5, collimated=1))
    W["witness"] = dict(n=256, z_centre=nz - 72.0 * L_l0, wake_cells=wake,
                        gamma_lab=2.0 / kp,
                        dephasing=(2 * math.pi / kp) ** 3 / LAMBDA0 ** 2)
    return W


# Laser entering a plasma in boosted frames approaching the group-velocity
# frame (the hyperbolic rotation of the laser's phase fronts, Fig. 2): lab
# density 1e-3 n_c starting 4 cells ahead of the box (knots: zero up to the
# lab position gamma_b dz (nz + 4), rising to n over 8 cells), gamma_b = 0.5,
# 0.7, 0.85 gamma_g; a plane-wave pulse (a0 = 0.1, L = 10 lambda0, uniform
# across a periodic 16-cell slab) at the box centre, in vacuum at t' = 0;
# 8192 cells along z at 16 per boosted vacuum wavelength, transverse cells of
# 16 lambda0, Courant number 0.99, current filter as in the energy-gain
# recipe (8 passes with compensation up to gamma_b = 16, 16 above), no
# window; the run lasts until the plasma has covered the pulse (0.37 box
# lengths of light travel).
BEATING_RATIOS = (0.5, 0.7, 0.85)


def time_beating(ratio, n=1e-3, passes=None, compensate=1):
    gb = ratio / math.sqrt(n)
    W = small("boost13_2d", nz=8192, nx=16, ppc=4, gamma_b=gb, n_lab=n, dx_lambda0=16.0,
              cfl=0.99, filter_passes=8 if gb <= 16.0 else 16, precision="fp32", window=None,
              laser=dict(a0=0.1, w0_lambda0=1.0e4, L_lambda0=10.0, place="box_center",
                         collimated=1))
    if passes is not None:
        W["filter_passes"] = passes
        W["filter_compensate"] = compensate
    W["plasma_start_cells"] = 4
    W["ramp_cells"] = 8
    W["travel_boxes"] = 0.37
    return W


# Laser guiding in a plasma channel, lab frame: a0 = 0.1 (linear), waist
# w0 = 8 lambda0 at the pulse centre, L = 4 lambda0, on-axis density 1e-3 n_c;
# 512 x 256 cells of lambda0/16 x lambda0/4 (32 x 64 lambda0, eight waists
# across), 2 pairs per cell, FP32, window at the group velocity, 1.5 Rayleigh
# lengths (pi w0^2 / lambda0) of propagation.  The matched channel's depth is
# the density rise 4 / (k0 w0)^2 n_c at r = w0, relative to the axis density.
def channel_guiding(matched=True):
    w0 = 8.0 * LAMBDA0
    n0 = 1e-3
    W = dict(
        dim=2, nz=512, nx=256, ny=1, gamma_b=1.0, dz_lambda0=1 / 16, dx_lambda0=0.25,
        cfl=0.95, n_lab=n0, ppc=2, order=1, filter_passes=1, filter_compensate=0, zbc="mur",
        precision="fp32", steps=None, seed=1017, window="group",
        laser=dict(a0=0.1, w0_lambda0=8.0, L_lambda0=4.0, place="front", front_gap=4.5,
                   collimated=1))
    W["channel"] = (4.0 / w0 ** 2 / n0, w0) if matched else None
    W["rayleigh"] = math.pi * w0 ** 2 / LAMBDA0
    W["propagation_rayleigh"] = 1.5
    return W


# One stage in plasma in the lab frame and in a frame boosted at gamma = 5,
# for their comparison in the lab frame (the lab-against-boost comparison of
# the section "Effect of the hyperbolic rotation in Minkowski space", Fig. 2).
#   * plasma: 0.01 n_c (k_p = 0.1) behind a 125 c/omega0 linear ramp, at rest
#     in the lab, ions as co-located partners; 2 pairs per cell at the cell
#     centres (a quiet start), a slab of 4 periodic transverse cells of
#     16 lambda0 (the problem is one-dimensional);
#   * laser: plane wave, a0 = 1, resonant Gaussian length L = sqrt(2) / k_p;
#   * numerics in both frames: `cells` cells per laser wavelength of the frame
#     (16 gamma_b (1 + beta_b) ... the Doppler-stretched one in the boosted
#     frame), CFL 0.95, 4 binomial passes with compensation, Mur ends, window
#     at the laser group velocity of the frame;
#   * placement: the boosted pulse is centred at z' = 2600 at t' = 0 and the
#     plasma front lies 200 c/omega0 beyond the pulse's leading cut (4 L'),
#     so that the whole t' = 0 field is a vacuum field; in lab coordinates the
#     plasma then starts at z_p = gamma_b z'_front.  The lab run starts at the
#     lab time T0 at which the pulse centre is 150 c/omega0 from the plasma
#     (row 0 of its window at lab z Z0, the pulse centre 290 above it) and runs
#     900 time units; the boosted run runs 2100 of its own;
#   * comparison grid (original lab coordinates): t from 50 after the pulse
#     centre meets the plasma, 280 samples 2 apart; zeta = z - v_g t from 300
#     behind the pulse centre, 720 samples 0.5 apart; the plasma front and its
#     transient have left that window from sample 240 on.
def lab_boost_pair(beta, boosted_dz, group_beta, yee_dt, cells=32):
    n0, a0, gb = 0.01, 1.0, 5.0
    kp = math.sqrt(n0)
    L = math.sqrt(2.0) / kp
    bb = beta(gb)
    dx, nx = 16.0 * LAMBDA0, 4
    ramp = 125.0
    scale = cells // 16
    dzb = boosted_dz(gb, LAMBDA0, cells)
    zL_b = 2600.0
    z_front_b = zL_b + 4.0 * L * gb * (1.0 + bb) + 200.0
    z_p = gb * z_front_b
    z_c = zL_b / (gb * (1.0 + bb))
    vg = group_beta(1.0, n0)
    T0 = (z_p - 150.0) - z_c
    Z0 = (z_p - 150.0) - 290.0
    dzl = LAMBDA0 / cells
    boost = dict(gamma_b=gb, nz=1024 * scale, dz=dzb, z_center=z_c,
                 knots_z=[z_p, z_p + ramp, 1.0e7], knots_n=[0.0, n0, n0],
                 beta_window=group_beta(gb, n0),
                 steps=int(2100.0 / yee_dt(2, dzb, dx, 1.0, 0.95)), every=1,
                 t_shift=0.0, z_shift=0.0)
    lab = dict(gamma_b=1.0, nz=1024 * scale, dz=dzl, z_center=290.0,
               knots_z=[z_p - Z0, z_p - Z0 + ramp, 1.0e7], knots_n=[0.0, n0, n0],
               beta_window=vg, steps=int(900.0 / yee_dt(2, dzl, dx, 1.0, 0.95)), every=2,
               t_shift=T0, z_shift=Z0)
    tc = z_p - z_c
    zeta_pc = z_c + (1.0 - vg) * tc
    grid = dict(t0=tc + 50.0, dt=2.0, nt=280, zeta0=zeta_pc - 300.0, dzeta=0.5, nzeta=720,
                front_gone=240)
    return dict(n0=n0, a0=a0, L=L, nx=nx, dx=dx, ppc=2, cfl=0.95, passes=4, seed=77,
                v_window=vg, boost=boost, lab=lab, grid=grid)
