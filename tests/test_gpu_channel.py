"""GPU: the plasma channel (the guiding channel of the paper's 10 GeV stage,
last figure): density n(z) (1 + depth r^2 / radius^2) about the laser axis.

  * parity with the oracle's channel (``tests/test_channel_pins.py`` pins it):
    birth weights to 1e-14, and full FP64 runs (boosted 2D with window, 3D
    quadratic) at the field parity bar of 1e-5;
  * the adjoint's density gradient with a channel (the transverse factor
    enters every weight) against FP64 central differences at 1e-4;
  * physics: a linear Gaussian beam (w0 = 8 lambda0) in the matched channel
    (density rise 4 / (k0 w0)^2 n_c at r = w0) keeps its spot over 1.5
    Rayleigh lengths (rms width within 12%), while without the channel it
    diffracts as w0 sqrt(1 + (z / Z_R)^2), 1.80 w0 at 1.5 Z_R (checked within
    10%).  The rms width of E_y^2 across x is w / 2 for a Gaussian field of
    waist w.
"""
import math

import numpy as np
import pytest

import oracle as O
from workloads import (WORKLOADS, adjoint_setup, channel_guiding, resolve_gpu, resolve_oracle,
                       small)

pytestmark = pytest.mark.gpu

COMPS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1011_0917_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


CASES = {"2d": ("boost13_2d_small", (1.2, 60.0)), "3d": ("boost100_3d_small", (0.8, 40.0))}


@pytest.mark.parametrize("case", list(CASES))
def test_channel_matches_oracle(P, case):
    name, ch = CASES[case]
    W = WORKLOADS[name]
    print("case channel parity", name, flush=True)
    cfg, init, nst = resolve_gpu(W, precision="fp64")
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"],
                            channel=ch)
    pg = sim.particles()
    w0g = np.sort(pg["w"][pg["id"] >= 0])
    sim.pic_step(nst)
    dg = sim.diagnostics(lineout=True)
    fg = {c: sim.get_field(c).cpu().numpy() for c in COMPS}
    sim.close()
    kw, oinit = resolve_oracle(W)
    s = O.Sim(**kw)
    s.init(n_uniform=oinit["n_lab"], laser=oinit["laser"], channel=ch)
    w0o = np.sort(s.particles()["w"])
    assert len(w0g) == len(w0o)
    assert np.abs(w0g - w0o).max() <= 1e-14 * w0o.max()
    assert w0o.max() > 1.2 * w0o.min()  # the channel shapes the weights
    s.step(nst)
    do = s.diagnostics(lineout=True)
    for k in ("ue", "ub", "ukin"):
        assert abs(dg[k] - do[k]) <= 1e-5 * abs(do[k]), k
    assert dg["live"] == do["live"]
    for c in COMPS:
        fo = s.get_field(c)
        assert np.abs(fg[c] - fo).max() <= 1e-5 * max(np.abs(fo).max(), 1e-300), c


def test_adjoint_density_gradient_with_channel(P):
    print("case adjoint_2d_tiny with a channel", flush=True)
    W = WORKLOADS["adjoint_2d_tiny"]
    cfg, init, nst = resolve_gpu(W, precision="fp64", sort_interval=0)
    dt = P.yee_dt(2, cfg.dz, cfg.dx, 1.0, cfg.cfl)
    a = adjoint_setup(W, cfg.dz, P.beta, dt)
    ch = (1.5, 20.0)

    def run(kn, grad=False):
        sim = P.Simulation(cfg, capacity=init["capacity"])
        sim.init_boosted_plasma(init["gamma_b"], knots_z=a["knots_z"], knots_n=list(kn),
                                laser=init["laser"], channel=ch)
        L = sim.forward_loss(nst, a["interval"], a["window"][0], a["window"][1], a["box"])
        g = sim.adjoint(len(kn))[1] if grad else None
        sim.close()
        return L, g

    kn = np.array(a["knots_n"])
    _, dn = run(kn, grad=True)
    h = 1e-6
    fd = []
    for m in range(len(kn)):
        kp, km = kn.copy(), kn.copy()
        kp[m] *= 1 + h
        km[m] *= 1 - h
        fd.append((run(kp)[0] - run(km)[0]) / (2 * h * kn[m]))
    fd = np.array(fd)
    scale = np.abs(fd).max()
    assert np.abs(np.array(dn) - fd).max() <= 1e-4 * scale, (dn, fd)


def spot_rms(P, matched):
    W = channel_guiding(matched)
    cfg, init, _ = resolve_gpu(W)
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"],
                            channel=W["channel"])
    steps = int(W["propagation_rayleigh"] * W["rayleigh"] / sim.dt)

    def rms():
        ey = sim.get_field("Ey").cpu().numpy()[:, :, 0]
        p = (ey ** 2).sum(axis=0)
        x = (np.arange(W["nx"]) - W["nx"] / 2) * cfg.dx
        return math.sqrt((p * x ** 2).sum() / p.sum())

    s0 = rms()
    sim.pic_step(steps)
    d = sim.diagnostics()
    s1 = rms()
    sim.close()
    assert not d["nan_flag"]
    return s0, s1, steps


def test_matched_channel_guides_the_laser(P):
    w0 = 8.0 * 2 * math.pi
    print("case channel guiding", flush=True)
    g0, g1, steps = spot_rms(P, True)
    f0, f1, _ = spot_rms(P, False)
    expect = math.sqrt(1.0 + 1.5 ** 2)
    print(f"{steps} steps; rms/(w0/2): channel {g0 / (w0 / 2):.3f} -> {g1 / (w0 / 2):.3f}, "
          f"no channel {f0 / (w0 / 2):.3f} -> {f1 / (w0 / 2):.3f} (diffraction {expect:.3f})",
          flush=True)
    assert abs(g0 / (w0 / 2) - 1.0) < 0.05 and abs(f0 / (w0 / 2) - 1.0) < 0.05
    assert abs(g1 / g0 - 1.0) < 0.12
    assert abs(f1 / f0 / expect - 1.0) < 0.10
