"""Pins of the oracle's plasma channel (CPU): lab density n(z) times
1 + depth r^2 / radius^2, r the distance from the laser axis (the box centre).

With the centred load every birth sits at a cell centre, so the summed weight
of the initial plasma has a closed form: over the half-integer offsets
m = j + 1/2 - nx/2 from the axis, sum_j m^2 = nx (nx^2 - 1) / 12, and
  sum w = gamma_b n dV nz [nx + depth dx^2 nx (nx^2 - 1) / (12 radius^2)]   (2D)
with the y sum added in 3D.  A misplaced axis, a missing cell size or a
squared radius gone astray changes the sum.
"""
import numpy as np
import pytest

import oracle as O


def _sim(dim, nz, nx, ny, gamma_b=13.0):
    return O.Sim(dim=dim, nz=nz, nx=nx, ny=ny, dz=0.7, dx=0.9, dy=1.3, dt=0.3, order=1, zbc=0,
                 ppc=2, load=1, gamma_b=gamma_b)


@pytest.mark.parametrize("dim", [2, 3])
def test_channel_total_weight_closed_form(dim):
    nz, nx, ny = 6, 10, 8 if dim == 3 else 1
    n0, depth, R = 2e-3, 1.7, 3.1
    s = _sim(dim, nz, nx, ny)
    s.init(n_uniform=n0, channel=(depth, R))
    w = s.particles()["w"]
    c = s.cfg
    dV = c.dz * c.dx * (c.dy if dim == 3 else 1.0)
    sq = lambda n: n * (n * n - 1) / 12.0  # noqa: E731
    ncell = nx * ny
    extra = c.dx ** 2 * sq(nx) * ny + (c.dy ** 2 * sq(ny) * nx if dim == 3 else 0.0)
    expect = c.gamma_b * n0 * dV * nz * (ncell + depth * extra / R ** 2)
    assert len(w) == nz * ncell * c.ppc
    assert abs(w.sum() - expect) <= 1e-12 * expect


def test_channel_weight_grows_off_axis():
    s = _sim(2, 4, 12, 1)
    s.init(n_uniform=1e-3, channel=(2.0, 4.0))
    p = s.particles()
    r = np.abs(p["xe"] - 6.0) * s.cfg.dx
    order = np.argsort(r)
    assert np.all(np.diff(p["w"][order]) >= -1e-18)
    on_axis = p["w"][order[0]]
    assert np.allclose(p["w"], on_axis * (1.0 + 2.0 * r ** 2 / 16.0) / (1.0 + 2.0 * r[order[0]] ** 2 / 16.0))


def test_no_channel_is_depth_zero():
    a = _sim(2, 4, 8, 1)
    a.init(n_uniform=1e-3)
    b = _sim(2, 4, 8, 1)
    b.init(n_uniform=1e-3, channel=(0.0, 0.0))
    assert np.array_equal(a.particles()["w"], b.particles()["w"])


def test_channel_rejects_bad_shape():
    s = _sim(2, 4, 8, 1)
    with pytest.raises(AssertionError):
        s.init(n_uniform=1e-3, channel=(-0.5, 2.0))
    with pytest.raises(AssertionError):
        s.init(n_uniform=1e-3, channel=(0.5, 0.0))
