"""Pins of the oracle's diagnostics normalisations, its density profile and its
sort keys (CPU).

* Field energy U = 1/2 sum F^2 dV: a uniform field in a box of known volume,
  and a cosine mode whose square sums to half the node count.
* Kinetic energy U_kin = sum w (gamma - 1): momenta whose gamma is rational
  (1 + |u|^2 a perfect square), so the expected sum is exact arithmetic.
* Energy exchange: in a cold-plasma oscillation the field energy and the
  kinetic energy trade places; their sum stays flat to the time-centring
  error of the leapfrog while each swings fully.  A field energy that drops
  or doubles its 1/2 fails this.
* Density profile: knot values, midpoints, zero outside, agreement with
  numpy's piecewise-linear interpolation, and the total weight of a centred
  load, which equals the trapezoid integral of the profile over the lab
  birth span when no knot falls inside a cell.
* Sort keys: a table of co-moving tile-major keys worked out by hand.
"""
import math

import numpy as np
import pytest

import oracle as O


# --------------------------------------------------------------------------
# U_E, U_B: uniform fields and a cosine mode
# --------------------------------------------------------------------------
@pytest.mark.parametrize("zbc", [0, 1])
def test_field_energy_of_uniform_fields(zbc):
    nz, nx, dz, dx = 12, 10, 0.7, 0.3
    s = O.Sim(dim=2, nz=nz, nx=nx, dz=dz, dx=dx, dt=0.1, zbc=zbc)
    s.init()
    E0, B0 = 0.37, -1.9
    s.set_field("Ex", E0)   # integer z rows: nz (periodic) or nz + 1 (open)
    s.set_field("Ez", 2 * E0)  # half-integer z rows: nz in either case
    s.set_field("By", B0)   # half-integer z rows
    d = s.diagnostics()
    rows_int = nz if zbc == 0 else nz + 1
    expect_e = 0.5 * (E0 ** 2 * rows_int + (2 * E0) ** 2 * nz) * nx * dz * dx
    expect_b = 0.5 * B0 ** 2 * nz * nx * dz * dx
    assert d["ue"] == pytest.approx(expect_e, rel=1e-14)
    assert d["ub"] == pytest.approx(expect_b, rel=1e-14)


def test_field_energy_3d_cosine_mode():
    nz, nx, ny, dz, dx, dy = 8, 6, 4, 0.5, 0.25, 2.0
    s = O.Sim(dim=3, nz=nz, nx=nx, ny=ny, dz=dz, dx=dx, dy=dy, dt=0.1, zbc=0)
    s.init()
    i = np.arange(nz + 1)[:, None, None]
    A = 3.0 * np.cos(2 * np.pi * 2 * i / nz) * np.ones((nz + 1, nx, ny))
    s.set_field("Bz", A)
    d = s.diagnostics()
    # sum over one period of cos^2 of a non-zero harmonic is half the count
    expect = 0.5 * 9.0 * (nz * nx * ny / 2) * dz * dx * dy
    assert d["ub"] == pytest.approx(expect, rel=1e-13)
    assert d["ue"] == 0.0


# --------------------------------------------------------------------------
# U_kin: rational gammas
# --------------------------------------------------------------------------
def test_kinetic_energy_rational_gammas():
    # (u_x, u_y, u_z) with 1 + |u|^2 a perfect square: gamma = 5/4, 5/3, 13/5, 5, 5
    moms = [((0.75, 0.0, 0.0), 1.25), ((0.0, 0.0, 4.0 / 3.0), 5.0 / 3.0),
            ((0.0, 2.4, 0.0), 2.6), ((2.0, 2.0, 4.0), 5.0), ((-2.0, 4.0, -2.0), 5.0)]
    weights = [0.5, 2.0, 0.125, 3.0, 1.0]
    gamma_b = 1.25
    s = O.Sim(dim=2, nz=8, nx=8, dz=1.0, dx=1.0, dt=0.1, zbc=0, gamma_b=gamma_b)
    s.init()
    for k, ((ux, uy, uz), _), w in zip(range(5), moms, weights):
        s.add_pair(2.5, 1.5 + k, 0.0, uz, ux, uy, 2.5, 1.5 + k, 0.0, w, k)
    d = s.diagnostics()
    expect = sum(w * (g - 1.0) for (_, g), w in zip(moms, weights))
    expect_drift = sum(w * (g - gamma_b) for (_, g), w in zip(moms, weights))
    assert d["ukin"] == pytest.approx(expect, rel=1e-14)
    assert d["ukin_drift"] == pytest.approx(expect_drift, rel=1e-14)
    assert d["charge"] == -sum(weights)
    assert d["live"] == 5


def test_kinetic_energy_of_plasma_at_rest_is_zero():
    s = O.Sim(dim=2, nz=8, nx=8, dz=1.0, dx=1.0, dt=0.1, zbc=0, ppc=2, seed=3)
    s.init(n_uniform=0.02)
    assert s.diagnostics()["ukin"] == 0.0


def test_energy_exchange_in_cold_plasma_oscillation():
    """Uniform electrons with u_z = du over immobile ions: E_z and the velocity
    trade energy at omega_p.  The leapfrog holds u half a step from E, so the
    sum U_E + U_kin carries an O(omega_p dt) wiggle; with omega_p dt = 0.02 it
    stays within a few percent of the swing of either term."""
    nz = nx = 4
    s = O.Sim(dim=2, nz=nz, nx=nx, dz=1.0, dx=1.0, dt=0.02, zbc=0, gamma_b=1.0)
    s.init()
    du, pid = 1e-3, 0
    for i in range(nz):
        for j in range(nx):
            s.add_pair(i + 0.5, j + 0.5, 0.0, du, 0.0, 0.0, i + 0.5, j + 0.5, 0.0, 1.0, pid)
            pid += 1
    ue, uk = [], []
    for _ in range(400):  # about 1.3 plasma periods
        s.step(1)
        d = s.diagnostics()
        ue.append(d["ue"] + d["ub"])
        uk.append(d["ukin"])
    ue, uk = np.array(ue), np.array(uk)
    swing = ue.max() - ue.min()
    assert swing > 0.9 * (uk.max() - uk.min()) and swing > 0.9 * uk.max()
    tot = ue + uk
    assert tot.max() - tot.min() < 0.03 * swing
    # the kinetic energy at start is n V du^2 / 2 to second order in du
    assert uk.max() == pytest.approx(nz * nx * (math.sqrt(1 + du * du) - 1), rel=1e-2)


# --------------------------------------------------------------------------
# Density profile
# --------------------------------------------------------------------------
KZ = np.array([10.0, 25.0, 40.0, 41.5, 90.0, 200.0])
KN = np.array([0.0, 1e-3, 2.5e-3, 2.5e-3, 4e-4, 1.2e-3])


def _profile_sim(gamma_b=3.0, load=1, nz=40, ppc=1, seed=0):
    s = O.Sim(dim=2, nz=nz, nx=4, dz=1.5, dx=0.5, dt=0.2, zbc=1, ppc=ppc, load=load,
              seed=seed, gamma_b=gamma_b)
    s.init(knots_z=KZ, knots_n=KN)
    return s


def test_lab_density_at_knots_midpoints_and_outside():
    s = _profile_sim()
    for z, n in zip(KZ, KN):
        assert s.lab_density(z) == n
    for m in range(len(KZ) - 1):
        mid = 0.5 * (KZ[m] + KZ[m + 1])
        assert s.lab_density(mid) == pytest.approx(0.5 * (KN[m] + KN[m + 1]), rel=1e-15, abs=1e-20)
    for z in (KZ[0] - 1e-9, -5.0, KZ[-1] + 1e-9, 1e6):
        assert s.lab_density(z) == 0.0


def test_lab_density_matches_numpy_interp():
    s = _profile_sim()
    z = np.random.default_rng(21).uniform(0.0, 220.0, 2000)
    got = np.array([s.lab_density(v) for v in z])
    ref = np.interp(z, KZ, KN, left=0.0, right=0.0)
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-20)


def test_centred_load_total_weight_is_trapezoid_integral():
    """Knots on lab cell boundaries: the midpoint rule on each cell is exact
    for a linear segment, so sum w = dx * integral of n over the birth span."""
    gamma_b, nz, dz, dx = 2.0, 30, 1.5, 0.5
    cell_lab = gamma_b * dz  # lab length of one co-moving cell at t' = 0
    kz = np.array([3, 9, 14, 22, 27], dtype=np.float64) * cell_lab
    kn = np.array([0.0, 2e-3, 2e-3, 5e-4, 0.0])
    s = O.Sim(dim=2, nz=nz, nx=4, dz=dz, dx=dx, dt=0.2, zbc=1, ppc=2, load=1, gamma_b=gamma_b)
    s.init(knots_z=kz, knots_n=kn)
    w = s.particles()["w"]
    trapezoid = float(np.sum(0.5 * (kn[1:] + kn[:-1]) * np.diff(kz)))
    assert w.sum() == pytest.approx(4 * dx * trapezoid, rel=1e-13)


def test_random_load_weights_follow_profile_at_birth():
    gamma_b, ppc = 3.0, 4
    s = _profile_sim(gamma_b=gamma_b, load=0, ppc=ppc, seed=77)
    p = s.particles()
    c = s.cfg
    z_lab = gamma_b * p["ze"] * c.dz  # births at t' = 0 with no drift yet
    expect = gamma_b * np.interp(z_lab, KZ, KN, left=0.0, right=0.0) * c.dz * c.dx / ppc
    assert np.allclose(p["w"], expect, rtol=1e-13, atol=1e-22)
    assert np.count_nonzero(p["w"]) > len(p["w"]) // 2


def test_channel_factor_on_axis_and_off_axis():
    s = O.Sim(dim=3, nz=4, nx=10, ny=6, dz=1.0, dx=0.5, dy=2.0, dt=0.1, zbc=0, load=1)
    s.init(n_uniform=1e-3, channel=(0.8, 2.0))
    assert s.channel_factor(5.0, 3.0) == 1.0  # the axis: box centre in x and y
    # 3 cells off in x (1.5) and 1 cell off in y (2.0): r^2 = 6.25, / R^2 = 1.5625
    assert s.channel_factor(8.0, 4.0) == pytest.approx(1.0 + 0.8 * 1.5625, rel=1e-15)
    assert s.channel_factor(2.0, 2.0) == pytest.approx(1.0 + 0.8 * 1.5625, rel=1e-15)


# --------------------------------------------------------------------------
# Sort keys worked out by hand
# --------------------------------------------------------------------------
def _keyed(dim, zbc, pts, tiles, tz_min, ntz, nz=32, nx=64, ny=8):
    s = O.Sim(dim=dim, nz=nz, nx=nx, ny=ny, dz=1.0, dx=1.0, dy=1.0, dt=0.1, zbc=zbc)
    s.init()
    for k, (z, x, y) in enumerate(pts):
        s.add_pair(z, x, y, 0.0, 0.0, 0.0, z, x, y, 1.0, 100 + k)
    key, pid = s.sort_keys(*tiles, tz_min, ntz)
    assert list(pid) == [100 + k for k in range(len(pts))]
    return list(key), s


def test_sort_keys_hand_table_2d():
    # 32 x 64 cells, tiles 16 x 32: 2 tile columns, 512 cells per tile;
    # key = (tile_z * 2 + tile_x) * 512 + lz * 32 + lx
    pts = [(3.5, 40.2, 0),    # cell (3, 40): tile (0, 1), local (3, 8) -> 512 + 104
           (17.0, 0.0, 0),    # cell (17, 0): tile (1, 0), local (1, 0) -> 1024 + 32
           (31.99, 63.5, 0),  # cell (31, 63): tile (1, 1), local (15, 31) -> 1536 + 511
           (-0.5, -0.25, 0),  # cell (-1, 63): row clamped to 0; tile (0, 1), local (0, 31)
           (40.0, 5.0, 0)]    # cell (40, 5): row clamped to 31; tile (1, 0), local (15, 5)
    key, s = _keyed(2, 1, pts, (16, 32, 1), 0, 2)
    assert key == [616, 1056, 2047, 543, 1509]
    # tile rows starting one tile lower: every row index grows by 16
    key, _ = _keyed(2, 1, pts[:4], (16, 32, 1), -1, 3)
    assert key == [1536 + 104, 2048 + 32, 2560 + 511, 512 + 15 * 32 + 31]
    # a window shift moves particles down the grid but not in the co-moving lattice
    key0, s = _keyed(2, 1, pts[:3], (16, 32, 1), 0, 2)
    s.window_shift(2)
    assert list(s.sort_keys(16, 32, 1, 0, 2)[0]) == key0


def test_sort_keys_hand_table_3d_periodic():
    # 16 x 8 x 8 cells, tiles 8 x 8 x 8: one tile per z slab, 512 cells per tile;
    # key = tile_z * 512 + (lz * 8 + lx) * 8 + ly
    pts = [(9.5, 2.5, 7.5),   # tile 1, local (1, 2, 7) -> 512 + 87
           (-0.5, 0.5, 0.5),  # periodic z: row 15 -> tile 1, local (7, 0, 0) -> 512 + 448
           (0.0, 7.9, 3.2)]   # tile 0, local (0, 7, 3) -> 59
    key, _ = _keyed(3, 0, pts, (8, 8, 8), 0, 2, nz=16, nx=8, ny=8)
    assert key == [599, 960, 59]


# --------------------------------------------------------------------------
# The parallel particle loop sums the same currents in another order
# --------------------------------------------------------------------------
@pytest.mark.skipif(O.max_threads() < 2, reason="oracle built without OpenMP")
@pytest.mark.parametrize("dim", [2, 3])
def test_threaded_particle_loop_matches_serial(dim):
    from workloads import WORKLOADS, resolve_oracle, small
    if dim == 2:
        W = small("boost13_2d", nz=48, nx=64, steps=6)
    else:
        W = small("boost100_3d", nz=24, nx=16, ny=16, steps=6)
    out = []
    for nt in (1, 4):
        kw, init = resolve_oracle(W)
        s = O.Sim(**kw)
        s.set_threads(nt)
        s.init(n_uniform=init["n_lab"], laser=init["laser"])
        s.step(6)
        # one particle's current at a node is of order w / (cell area dt): the
        # electron and partner terms of a pair cancel to far below that, so
        # round-off of the order of addition is measured against it
        unit = s.particles()["w"].max() / (kw["dx"] * kw["dt"] * (kw["dy"] if dim == 3 else 1.0))
        out.append((s.diagnostics(lineout=True), s.get_field("Jz"), s.get_field("Ey"), unit))
    (d1, j1, e1, unit), (d4, j4, e4, _) = out
    for k in ("ue", "ub", "ukin"):
        assert d4[k] == pytest.approx(d1[k], rel=1e-12)
    assert d4["live"] == d1["live"]
    assert np.abs(j4 - j1).max() <= 1e-14 * unit
    assert np.abs(e4 - e1).max() <= 1e-12 * np.abs(e1).max()
