"""Pins of the oracle's witness electrons (CPU).

The gather by exactness on linear fields (linear and quadratic shapes
reproduce a linear function, so a wrong node offset or weight shows), with the
Yee node offsets written out here on their own; gather, push and move
together against the oracle's own particle step (a zero-weight plasma pair
leaves the fields alone, and its electron sees the same start-of-step fields),
in open and periodic z, with positions at the periodic seam; the push by the closed forms of a uniform electric field (u changes by -E dt per
step, exactly, in the Boris step) and of a uniform magnetic field (|u| is
conserved and the momentum turns by 2 atan(B dt / (2 gamma)) per step); the
lab view by a witness at rest in the calculation frame (gamma = gamma_b,
u_z = gamma_b beta_b) and by the invariance of gamma^2 - u^2 = 1.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import witness as WT


# Yee lattice: E_a on the edges along a, B_a on the faces normal to a
# (offsets in cells along z, x, y)
YEE_NODES = {"Ex": (0.0, 0.5, 0.0), "Ey": (0.0, 0.0, 0.5), "Ez": (0.5, 0.0, 0.0),
             "Bx": (0.5, 0.0, 0.5), "By": (0.5, 0.5, 0.0), "Bz": (0.0, 0.5, 0.5)}


def _sim(dim=2, order=1, nz=24, nx=16, ny=1, zbc=1):
    s = O.Sim(dim=dim, nz=nz, nx=nx, ny=ny, dz=0.7, dx=0.9, dy=1.1, dt=0.3, order=order, zbc=zbc)
    s.init()
    return s


@pytest.mark.parametrize("dim,order", [(2, 1), (3, 2)])
def test_gather_exact_on_linear_fields(dim, order):
    s = _sim(dim=dim, order=order, ny=12 if dim == 3 else 1)
    c = s.cfg
    rng = np.random.default_rng(5)
    coef = {}
    for name, (sz, sx, sy) in YEE_NODES.items():
        a, bz, bx = rng.uniform(-1, 1, 3)
        coef[name] = (a, bz, bx)
        i = np.arange(c.nz + 1)[:, None, None] + sz
        j = np.arange(c.nx)[None, :, None] + sx
        s.set_field(name, np.broadcast_to(a + bz * i + bx * j, s.shape))
    F = WT.fields(s)
    for z, x, y in [(8.3, 5.6, 4.2), (12.9, 7.05, 6.5), (10.0, 6.5, 5.0)]:
        E, B = WT.gather(F, s, z, x, y)
        got = dict(zip(["Ex", "Ey", "Ez", "Bx", "By", "Bz"], E + B))
        for name, (a, bz, bx) in coef.items():
            assert abs(got[name] - (a + bz * z + bx * x)) < 1e-12, name


@pytest.mark.parametrize("dim,order,zbc", [(2, 1, 1), (2, 2, 0), (3, 1, 0), (3, 2, 1)])
def test_push_matches_oracle_particle_step(dim, order, zbc):
    s = _sim(dim=dim, order=order, ny=10 if dim == 3 else 1, zbc=zbc)
    c = s.cfg
    rng = np.random.default_rng(17 + dim + order + zbc)
    for name in YEE_NODES:
        a = rng.uniform(-0.5, 0.5, s.shape)
        if zbc == 0:
            a[c.nz] = 0.0
        s.set_field(name, a)
    zs = [0.15, c.nz - 0.3, 0.6] if zbc == 0 else [5.2, 11.7, 17.05]
    W = np.array([[z, rng.uniform(0, c.nx), rng.uniform(0, c.ny) if dim == 3 else 0.0,
                   *rng.uniform(-2, 2, 3)] for z in zs])
    for r in W:
        s.add_pair(r[0], r[1], r[2], r[3], r[4], r[5], r[0], r[1], r[2], 0.0, 0)
    WT.push(s, W)
    s.step(1)
    p = s.particles()
    got = np.stack([p["ze"], p["xe"], p["ye"], p["uz"], p["ux"], p["uy"]], axis=1)
    assert np.abs(got - W).max() < 1e-13


def test_uniform_electric_field_closed_form():
    s = _sim()
    E0 = 0.37
    s.set_field("Ex", np.full(s.shape, E0))
    W = np.array([[10.2, 4.3, 0.0, 0.1, 0.2, -0.3]])
    for n in range(1, 41):
        WT.push(s, W)
        assert abs(W[0, 4] - (0.2 - n * s.cfg.dt * E0)) < 1e-12
        assert W[0, 3] == 0.1 and W[0, 5] == -0.3


def test_uniform_magnetic_field_rotation():
    s = _sim()
    B0 = 0.8
    s.set_field("Bz", np.full(s.shape, B0))
    W = np.array([[10.2, 4.3, 0.0, 0.0, 0.6, 0.0]])
    u0 = math.hypot(W[0, 4], W[0, 5])
    g = math.sqrt(1 + u0 * u0)
    th = 2 * math.atan(B0 * s.cfg.dt / (2 * g))
    phase0 = math.atan2(W[0, 5], W[0, 4])
    for n in range(1, 30):
        WT.push(s, W)
        assert abs(math.hypot(W[0, 4], W[0, 5]) - u0) < 1e-14
        ph = math.atan2(W[0, 5], W[0, 4])
        # q = -1: the momentum turns by +th about +z per step
        assert abs(math.remainder(ph - phase0 - n * th, 2 * math.pi)) < 1e-12


def test_lab_view_invariants():
    g = 13.0
    b = O.beta_of_gamma(g)
    W = np.array([[3.0, 1.0, 0.0, 0.0, 0.0, 0.0], [5.0, 2.0, 0.0, 4.0, -1.5, 0.7]])
    out = WT.lab(W, t_prime=2.0, window_cells=1.0, dz=0.5, gamma_b=g)
    assert abs(out[0, 2] - g) < 1e-12 and abs(out[0, 3] - g * b) < 1e-12
    for r in range(len(W)):
        assert abs(out[r, 2] ** 2 - out[r, 3] ** 2 - W[r, 4] ** 2 - W[r, 5] ** 2 - 1.0) < 1e-9
    # a witness at z' = 0 at t' = 0 sits at the lab origin
    z0 = WT.lab(np.array([[-1.0, 0, 0, 0, 0, 0]]), 0.0, 1.0, 0.5, g)
    assert abs(z0[0, 0]) < 1e-15 and abs(z0[0, 1]) < 1e-15
