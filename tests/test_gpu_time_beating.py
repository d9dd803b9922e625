"""GPU: the boosted laser as the frame approaches the laser group velocity
(section "Effect of the hyperbolic rotation in Minkowski space", Fig. 2).

A pulse launched in vacuum enters a plasma of lab density n.  The lab
frequency is kept (the plasma is at rest in the lab), so inside the plasma the
lab wave has omega_0 = 1 and k = sqrt(1 - n); in the frame moving at beta_b
its wavenumber and frequency are
    k' = gamma_b (k - beta_b),   omega' = gamma_b (1 - beta_b k).
Against the vacuum values gamma_b (1 - beta_b), with gamma_g = n^-1/2,
    k' / k'_vac -> 1 - gamma_b^2 / gamma_g^2,  omega' / omega'_vac -> 1 + gamma_b^2 / gamma_g^2
(to order n): as gamma_b -> gamma_g the phase fronts turn until the field
oscillates in time with hardly any variation in space, the time beating of
the paper.  Checked at gamma_b / gamma_g = 0.5, 0.7, 0.85 (recipe:
``workloads.time_beating``):
  * at t' = 0 (vacuum) the spectral peak of the on-axis record sits at k'_vac
    within one bin;
  * the on-axis field at the pulse's centre row oscillates in time at the
    closed-form omega' within 3% (observed: within 1.1%);
  * (second test) frames nearer gamma_g tolerate more filtering at the same
    accuracy, the key finding of section "Mitigation of a numerical
    instability": the current filter scales the plasma's response at the
    laser's boosted wavenumber by its transfer T(k'), so the lab wave sees
    n T and omega' = gamma_b (1 - beta_b sqrt(1 - n T)), with k' = gamma_b
    (sqrt(1 - n T) - beta_b) found self-consistently.  For 16 plain binomial
    passes (T = cos^32(k' dz / 2)) the plasma response loses 35% at
    gamma_b / gamma_g = 0.5 but 6% at 0.85, where the laser's boosted
    wavelength spans 50 cells instead of 19.  Checked: omega' against that
    closed form within 3%, and the loss at 0.85 below a third of that at 0.5;
  * once the plasma covers the pulse, the peak wavenumber falls
    monotonically with gamma_b and follows the closed form within
    0.06 k'_vac.  k' is a small difference, gamma_b (k - beta_b): a relative
    error d of the grid's phase velocity in the plasma moves it by about
    2 gamma_b^2 d k'_vac, so 3e-5 of Yee and plasma dispersion becomes
    0.04 k'_vac at gamma_b = 27 (observed: 0.002 to 0.042, depending on the
    filtering), where omega' is no such difference.
"""
import math

import numpy as np
import pytest

from workloads import BEATING_RATIOS, resolve_gpu, time_beating

pytestmark = pytest.mark.gpu

M = 8192
NT = 256


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1011_0917_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def run(P, ratio, **filt):
    W = time_beating(ratio, **filt)
    nz = W["nz"]
    cfg, init, _ = resolve_gpu(W, capacity=nz * W["nx"] * W["ppc"] * 2 + 100000)
    gb, dz = init["gamma_b"], cfg.dz
    zs = gb * dz * (nz + W["plasma_start_cells"])
    kz = [0.0, zs, zs + gb * dz * W["ramp_cells"], zs + gb * dz * 1.0e6]
    kn = [0.0, 0.0, W["n_lab"], W["n_lab"]]
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(gb, knots_z=kz, knots_n=kn, laser=init["laser"])
    r0, _ = sim.axis_record(0)
    p0 = sim.axis_spectrum(r0[None, :M], M).cpu().numpy()[0]
    u0 = sim.diagnostics()
    u0 = u0["ue"] + u0["ub"]
    steps = int(W["travel_boxes"] * nz * dz / sim.dt)
    sim.pic_step(steps)
    r1, _ = sim.axis_record(0)
    p1 = sim.axis_spectrum(r1[None, :M], M).cpu().numpy()[0]
    row = int(np.argmax(np.abs(r1.cpu().numpy())))
    hist = np.empty(NT)
    for t in range(NT):
        sim.pic_step(1)
        hist[t] = float(sim.axis_record(0)[0][row])
    d = sim.diagnostics()
    d["u0"] = u0
    sim.close()
    return gb, dz, sim.dt, p0, p1, hist, d


def peak_frequency(x, dt):
    """Angular frequency of the spectral peak of a Hann-windowed series,
    zero-padded to 64x its length, with a parabolic fit through the peak."""
    n = len(x)
    X = np.abs(np.fft.rfft((x - x.mean()) * np.hanning(n), 64 * n))
    k = int(np.argmax(X[1:])) + 1
    a, b, c = X[k - 1], X[k], X[k + 1]
    k += 0.5 * (a - c) / (a - 2 * b + c)
    return 2 * math.pi * k / (64 * n * dt)


def test_boosted_laser_turns_into_a_time_beating(P):
    n = time_beating(0.5)["n_lab"]
    last = None
    for ratio in BEATING_RATIOS:
        print("case time beating, gamma_b / gamma_g =", ratio, flush=True)
        gb, dz, dt, p0, p1, hist, d = run(P, ratio)
        assert not d["nan_flag"]
        bb = P.beta(gb)
        kvac = gb * (1.0 - bb)
        k = math.sqrt(1.0 - n)
        kp, wp = gb * (k - bb), gb * (1.0 - bb * k)
        q = lambda kk: kk * M * dz / (2 * math.pi)  # noqa: E731
        q0 = int(np.argmax(p0[1:])) + 1
        q1 = int(np.argmax(p1[1:])) + 1
        w = peak_frequency(hist, dt)
        print(f"k'/k'_vac: measured {q1 / q(kvac):.3f}, closed form {kp / kvac:.3f}; "
              f"omega'/omega'_vac: measured {w / kvac:.3f}, closed form {wp / kvac:.3f}; "
              f"field energy {d['u0']:.3e} -> {d['ue'] + d['ub']:.3e}", flush=True)
        assert abs(q0 - q(kvac)) <= 1.0
        assert abs(w / wp - 1.0) < 0.03
        assert abs(q1 - q(kp)) <= 0.06 * q(kvac)
        if last is not None:
            assert q1 < last
        last = q1


def filtered_transfer(n, gb, bb, dz, passes):
    """Self-consistent transfer T of `passes` plain binomial passes at the
    boosted wavenumber of the wave in a plasma seen through that filter."""
    T = 1.0
    for _ in range(100):
        kp = gb * (math.sqrt(1.0 - n * T) - bb)
        T = math.cos(0.5 * kp * dz) ** (2 * passes)
    return T


def test_higher_boost_tolerates_more_filtering(P):
    n = time_beating(0.5)["n_lab"]
    loss = {}
    for ratio in (0.5, 0.85):
        print("case filtering tolerance, gamma_b / gamma_g =", ratio, flush=True)
        gb, dz, dt, _, _, hist, d = run(P, ratio, passes=16, compensate=0)
        assert not d["nan_flag"]
        bb = P.beta(gb)
        wvac = gb * (1.0 - bb)
        T = filtered_transfer(n, gb, bb, dz, 16)
        w_true = gb * (1.0 - bb * math.sqrt(1.0 - n))
        w_filt = gb * (1.0 - bb * math.sqrt(1.0 - n * T))
        w = peak_frequency(hist, dt)
        loss[ratio] = 1.0 - (w - wvac) / (w_true - wvac)
        print(f"omega'/omega'_vac: measured {w / wvac:.3f}, filtered closed form "
              f"{w_filt / wvac:.3f}, unfiltered {w_true / wvac:.3f}; plasma response lost "
              f"{loss[ratio]:.3f} (closed form {1.0 - T:.3f})", flush=True)
        assert abs(w / w_filt - 1.0) < 0.03
    assert loss[0.85] < loss[0.5] / 3.0
