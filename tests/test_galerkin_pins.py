"""Pins of the oracle's energy-conserving (Galerkin) gather (CPU).

In the Galerkin form a field component takes, along each axis on which it
sits at half-integer nodes, the shape of one order lower than the deposit's:
nearest half node (order 0) for linear particles, linear for quadratic ones.
What fixes it:

* order-0 shape: a partition of unity with exactly one node, the one whose
  half-open cell [i - 1/2, i + 1/2) holds the point;
* a field that is linear in position is reproduced exactly along every axis
  of full order, and along a reduced axis of a linear-shape run it is read at
  the half node of the particle's cell (piecewise constant), of a quadratic
  run exactly (linear shapes reproduce linear functions);
* with the same shape on every axis the form reduces to the momentum-
  conserving gather (a field constant along its staggered axes gathers alike);
* energy: a warm plasma whose Debye length is a twentieth of a cell heats
  numerically under the momentum-conserving gather (the finite-grid
  instability), while the energy-conserving gather holds the total energy
  (Birdsall and Langdon, the energy-conserving algorithms).
"""
import math

import numpy as np
import pytest

import oracle as O

STAG = {"Ex": (0, .5, 0), "Ey": (0, 0, .5), "Ez": (.5, 0, 0)}


def test_order0_shape_is_nearest_grid_point():
    rng = np.random.default_rng(4)
    for xi in rng.uniform(-4, 4, 200):
        w = np.array([O.shape(0, xi - i) for i in range(-6, 7)])
        assert w.sum() == 1.0 and np.count_nonzero(w) == 1
        assert -6 + int(np.argmax(w)) == math.floor(xi + 0.5)
    # the half-open cell: a point half-way between nodes belongs to the upper one
    assert O.shape(0, -0.5) == 1.0 and O.shape(0, 0.5) == 0.0


def _gathered_e(dim, order, comp, f_of, zp, xp, yp, gather):
    """u after one step of a w = 0 electron at rest under E alone: -dt E(particle)."""
    nz, nx, ny = (12, 10, 10) if dim == 3 else (12, 10, 1)
    dz, dx, dy, dt = 0.8, 0.6, 0.7, 0.1
    sz, sx, sy = STAG[comp]
    s = O.Sim(dim=dim, nz=nz, nx=nx, ny=ny, dz=dz, dx=dx, dy=dy, dt=dt, order=order, zbc=1,
              ions=0, gather=gather)
    s.init()
    i, j, l = np.meshgrid(np.arange(nz + 1), np.arange(nx), np.arange(ny if dim == 3 else 1),
                          indexing="ij")
    s.set_field(comp, f_of((i + sz) * dz, (j + sx) * dx, (l + sy) * dy))
    s.add_pair(zp, xp, yp, 0.0, 0.0, 0.0, zp, xp, yp, 0.0, 0)
    s.step(1)
    p = s.particles()
    u = {"Ex": p["ux"][0], "Ey": p["uy"][0], "Ez": p["uz"][0]}[comp]
    return -u / dt, (dz, dx, dy)


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_linear_fields_on_reduced_and_full_axes(dim, order):
    a, bz, bx, by = 0.3, 0.05, -0.04, 0.07
    f = lambda z, x, y: a + bz * z + bx * x + (by * y if dim == 3 else 0.0)  # noqa: E731
    for zp, xp, yp in ((5.37, 4.81, 4.23), (6.62, 3.12, 5.71), (5.5, 4.5, 4.5)):
        for comp, (sz, sx, sy) in STAG.items():
            if dim == 2 and comp == "Ey":
                sy = 0.0  # no y axis in 2D: every in-plane axis has full order
            got, (dz, dx, dy) = _gathered_e(dim, order, comp, f, zp, xp, yp, 1)
            # position read along each axis: the true one, or on a reduced
            # axis of a linear-shape run the half node of the particle's cell
            def read(p, s_):
                return math.floor(p) + 0.5 if (s_ == 0.5 and order == 1) else p
            expect = f(read(zp, sz) * dz, read(xp, sx) * dx, read(yp, sy) * dy)
            assert abs(got - expect) < 1e-14, (comp, got, expect)


def test_uniform_field_along_staggered_axes_gathers_like_momentum_form():
    """A field that varies only across its own staggered axes is read the same
    by both forms (the reduced shape matters only where the field varies)."""
    f = lambda z, x, y: 0.4 - 0.03 * x  # noqa: E731 -- varies along x only
    got1, _ = _gathered_e(2, 1, "Ez", f, 5.37, 4.81, 0.0, 1)
    got0, _ = _gathered_e(2, 1, "Ez", f, 5.37, 4.81, 0.0, 0)
    assert abs(got1 - got0) < 1e-15


def _magnetic_rotation(order, gather, zp, xp):
    """By linear in z and x, sampled on its (1/2, 1/2) lattice: one Boris step
    rotates u about y by 2 atan(|q| By(read) dt / (2 gamma))."""
    nz, nx, dz, dx, dt = 12, 10, 0.8, 0.6, 0.2
    s = O.Sim(dim=2, nz=nz, nx=nx, dz=dz, dx=dx, dt=dt, order=order, zbc=1, ions=0,
              gather=gather)
    s.init()
    i, j = np.meshgrid(np.arange(nz + 1), np.arange(nx), indexing="ij")
    s.set_field("By", (0.8 + 0.06 * (i + 0.5) * dz - 0.05 * (j + 0.5) * dx)[..., None])
    u0 = np.array([0.3, 0.0, 0.4])
    s.add_pair(zp, xp, 0.0, u0[2], u0[0], u0[1], zp, xp, 0.0, 0.0, 0)
    s.step(1)
    p = s.particles()
    g = math.sqrt(1 + u0 @ u0)
    ang = math.atan2(p["uz"][0], p["ux"][0]) - math.atan2(u0[2], u0[0])
    return abs(ang), g, dz, dx, dt


@pytest.mark.parametrize("order", [1, 2])
def test_magnetic_field_read_on_reduced_axes(order):
    zp, xp = 5.61, 4.27
    ang, g, dz, dx, dt = _magnetic_rotation(order, 1, zp, xp)
    rz, rx = (math.floor(zp) + 0.5, math.floor(xp) + 0.5) if order == 1 else (zp, xp)
    By = 0.8 + 0.06 * rz * dz - 0.05 * rx * dx
    assert abs(ang - 2 * math.atan(By * dt / (2 * g))) < 1e-14


def _warm_plasma_energy(gather, order, n=16, ppc=16, vth=0.05, steps=600, dt=0.1, seed=3):
    s = O.Sim(dim=2, nz=n, nx=n, dz=1.0, dx=1.0, dt=dt, order=order, zbc=0, gamma_b=1.0,
              gather=gather)
    s.set_threads(min(4, max(1, O.max_threads())))
    s.init()
    rng = np.random.default_rng(seed)
    pid = 0
    for i in range(n):
        for j in range(n):
            for _ in range(ppc):
                z, x = i + rng.random(), j + rng.random()
                u = rng.normal(0.0, vth, 3)
                s.add_pair(z, x, 0.0, u[2], u[0], u[1], z, x, 0.0, 1.0 / ppc, pid)
                pid += 1
    d0 = s.diagnostics()
    s.step(steps)
    d1 = s.diagnostics()
    e0 = d0["ue"] + d0["ub"] + d0["ukin"]
    e1 = d1["ue"] + d1["ub"] + d1["ukin"]
    return (e1 - e0) / e0


def test_energy_conserving_gather_holds_a_cold_grid_plasma():
    """Electrons of density 1 (omega_p = 1) at v_th = 0.05 c on unit cells
    (Debye length dx / 20), ions immobile, 60 plasma times: the
    momentum-conserving linear gather heats the plasma by a third of its
    energy, the energy-conserving one keeps the total within 0.2 %."""
    heat_mc = _warm_plasma_energy(0, 1)
    heat_ec = _warm_plasma_energy(1, 1)
    assert heat_mc > 0.1, heat_mc
    assert abs(heat_ec) < 2e-3, heat_ec
