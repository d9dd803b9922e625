"""Pins of the oracle's lab-frame and spectral diagnostics (CPU).

The back transform is pinned by a function it must reproduce exactly (linear
in t' and z': linear interpolation is exact) and by the invariance of a plane
wave's phase, k0 (z - t) = k' (z' - t') with k' = gamma (1 - beta) k0; the
field transform by the lab field of a boosted plane wave; the spectrum by a
pure cosine and Parseval's relation; the boosted laser of the oracle's own
init by the plane-wave transform of the carrier (E' = gamma (1 - beta) E,
k' = gamma (1 - beta) k0).
"""
import math

import numpy as np

import oracle as O
from oracle import labframe as LF
from workloads import LAMBDA0, WORKLOADS, resolve_oracle


def test_back_transform_exact_for_linear_history():
    rng = np.random.default_rng(7)
    g = 5.0
    b = O.beta_of_gamma(g)
    n, nrec, dz = 40, 9, 0.7
    tp = np.cumsum(rng.uniform(0.5, 1.5, nrec))          # uneven record times
    z0 = np.floor(rng.uniform(0, 3, nrec)) * dz          # window offsets
    a0, az, at = 0.3, -1.7, 2.9
    rec = np.array([[a0 + az * (z0[r] + i * dz) + at * tp[r] for i in range(n)]
                    for r in range(nrec)])
    # recorded: t' in [~1, ~9], z' in [0, ~30]; seen through a window moving
    # at 0.9: t = gamma (t' + beta z') in [0, ~180], zeta = z - 0.9 t in [0, ~20]
    t0, dt, nt, zeta0, dzeta, nz_ = 0.0, 5.0, 40, -2.0, 0.4, 60
    out = LF.back_transform(rec, tp, z0, dz, g, t0, dt, nt, zeta0, dzeta, nz_, 0.9)
    fin = np.isfinite(out)
    assert fin.sum() > 50 and (~fin).sum() > 50
    for m, k in zip(*np.nonzero(fin)):
        t = t0 + m * dt
        z = zeta0 + k * dzeta + 0.9 * t
        tpe, zpe = g * (t - b * z), g * (z - b * t)
        assert abs(out[m, k] - (a0 + az * zpe + at * tpe)) < 1e-9


def test_back_transform_plane_wave_phase_invariant():
    """Records of cos(k' (z' - t')) back-transformed give cos(k0 (z - t))."""
    g = 5.0
    b = O.beta_of_gamma(g)
    kp = 1.0 * g * (1.0 - b)
    lam_p = 2 * math.pi / kp
    dz = lam_p / 256
    n = 600
    tp = np.arange(0, 40) * (lam_p / 256)
    rec = np.array([[math.cos(kp * (i * dz - t)) for i in range(n)] for t in tp])
    # recorded: z' in [0, ~146], t' in [0, ~9.5], i.e. lab t up to ~760 and
    # zeta = z - t = gamma (1 - beta) (z' - t') up to ~14
    out = LF.back_transform(rec, tp, np.zeros(len(tp)), dz, g, 0.0, 25.0, 30, 0.0, 0.035, 400,
                            1.0)
    fin = np.isfinite(out)
    assert fin.sum() > 100
    err = 0.0
    for m, k in zip(*np.nonzero(fin)):
        zeta = 0.035 * k
        err = max(err, abs(out[m, k] - math.cos(zeta)))   # z - t = zeta, k0 = 1
    # linear interpolation in z' and t' on 256 points per wavelength
    assert err < 2 * (2 * math.pi / 256) ** 2 / 8 + 1e-12


def _vacuum_sim(name="lab_history_2d"):
    W = WORKLOADS[name]
    kw, init = resolve_oracle(W)
    s = O.Sim(**kw)
    s.init(laser=init["laser"])
    return W, kw, init, s


def test_record_lab_field_of_boosted_plane_wave():
    """Fields set to the boosted image of the lab wave E_y = -B_x = cos(k0 (z - t))
    at t' = 0: frame 0 returns E'_y, frame 1 the lab wave at the same events."""
    W, kw, _, s = _vacuum_sim()
    g, b = kw["gamma_b"], O.beta_of_gamma(kw["gamma_b"])
    d = g * (1 - b)
    dz = kw["dz"]
    nz, nx = kw["nz"], kw["nx"]
    z = np.arange(nz + 1) * dz
    ey = np.repeat((d * np.cos(d * z))[:, None, None], nx, axis=1)
    bx = np.repeat((-d * np.cos(d * (z + 0.5 * dz)))[:, None, None], nx, axis=1)
    bx[nz] = 0.0
    s.set_field("Ey", ey)
    s.set_field("Bx", bx)
    r0 = LF.record(s, 0, g)
    r1 = LF.record(s, 1, g)
    assert np.abs(r0 - d * np.cos(d * z)).max() < 1e-14
    # the lab field at z = gamma z', t = gamma beta z' is cos(gamma (1 - beta) z');
    # B'_x averaged onto the node carries cos(k' dz / 2)
    lab = np.cos(d * z)[1:nz]
    assert np.abs(r1[1:nz] - lab).max() < 0.5 * (d * dz) ** 2 / 4 + 1e-12


def test_spectrum_cosine_and_parseval():
    m = 256
    q0 = 19
    x = np.cos(2 * math.pi * q0 * np.arange(m) / m)
    p = LF.spectrum(x, m)[0]
    assert abs(p[q0] - (m / 2) ** 2) < 1e-9
    assert np.delete(p, q0).max() < 1e-18 * m * m + 1e-16
    rng = np.random.default_rng(3)
    y = rng.standard_normal(100)
    p = LF.spectrum(y, m)[0]
    parseval = (p[0] + 2 * p[1:m // 2].sum() + p[m // 2]) / m
    assert abs(parseval - (y ** 2).sum()) < 1e-10 * (y ** 2).sum()


def test_boosted_laser_carrier_transform():
    """The oracle's boosted laser at t' = 0: its on-axis E'_y peaks at
    gamma (1 - beta) a0 and its spectrum at k' = gamma (1 - beta) k0."""
    W, kw, init, s = _vacuum_sim()
    g, b = kw["gamma_b"], O.beta_of_gamma(kw["gamma_b"])
    d = g * (1 - b)
    r0 = LF.record(s, 0, g)
    a0 = W["laser"]["a0"]
    assert abs(np.abs(r0).max() / (d * a0) - 1.0) < 0.02
    m = 4096
    p = LF.spectrum(r0, m)[0]
    q_peak = int(np.argmax(p))
    q_carrier = d * 1.0 * m * kw["dz"] / (2 * math.pi)   # k0 = 1 (units of omega0 / c)
    assert abs(q_peak - q_carrier) <= 1.0, (q_peak, q_carrier)
    assert LAMBDA0 == 2 * math.pi


def test_vacuum_history_reproduces_lab_pulse():
    W, kw, init, s = _vacuum_sim()
    g = kw["gamma_b"]
    dt = kw["dt"]
    recs, tps = [LF.record(s, 1, g)], [0.0]
    for n in range(W["steps"]):
        s.step(1)
        recs.append(LF.record(s, 1, g))
        tps.append((n + 1) * dt)
    grid = (900.0, 40.0, 100, 0.0, 0.2, 500, 1.0)
    out = LF.back_transform(np.array(recs), np.array(tps), np.zeros(len(tps)), kw["dz"], g, *grid)
    fin = np.isfinite(out)
    assert fin.sum() > 1000
    t0, dtl, nt, zeta0, dzeta, nzeta, vw = grid
    lab = np.array([O.laser_eval(init["laser"], 2, 1.0, zeta0 + k * dzeta + vw * (t0 + m * dtl),
                                 0.0, tp=t0 + m * dtl)[1] for m, k in zip(*np.nonzero(fin))])
    err = np.linalg.norm(out[fin] - lab) / np.linalg.norm(lab)
    assert err < 0.06, err
