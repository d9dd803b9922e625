"""GPU: the laser antenna (``bfpic_antenna``) against the oracle's.

* FP64 element by element at 1e-5 against the FP64 oracle with the same
  antenna: a boosted 2D run with plasma and moving window (gamma_b = 13) and a
  3D quadratic run (gamma_b = 100), each with the pulse init placed in the
  box and an antenna whose pulse has its centre at the antenna row at mid-run;
  the antenna's field (the oracle's difference from a run without it) must
  exceed half the target amplitude at the antenna;
* the emitted pulse against the analytic one (FP32, gamma_b = 5, vacuum,
  32 cells per wavelength): within 5% in L2, the bound the oracle's own pin
  holds (observed 3.0% there);
* error paths: a row outside 1 .. nz-1, an antenna before init, and a taped
  adjoint run with an antenna.
"""
import math

import numpy as np
import pytest

import oracle as O
from workloads import WORKLOADS, resolve_gpu, resolve_oracle

pytestmark = pytest.mark.gpu

COMPS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")
LAMBDA0 = 2.0 * math.pi


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1011_0917_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def _antenna_laser(W, dz, row, beta, t_mid):
    """The workload's laser, its centre crossing the antenna row (in the
    frame) at t' = t_mid."""
    g = W["gamma_b"]
    dop = 1.0 / (g * (1.0 + beta(g)))
    zc = row * dz - t_mid
    return dict(a0=W["laser"]["a0"], w0=W["laser"]["w0_lambda0"] * LAMBDA0,
                L=W["laser"]["L_lambda0"] * LAMBDA0, z_center=dop * zc, z_focus=g * zc,
                collimated=W["laser"].get("collimated", 0))


@pytest.mark.parametrize("name,row", [("boost13_2d_small", 24), ("boost100_3d_small", 8)])
def test_antenna_fp64_matches_oracle(P, name, row):
    W = WORKLOADS[name]
    print("case antenna fp64", name, flush=True)
    cfg, init, nst = resolve_gpu(W, precision="fp64")
    sim = P.Simulation(cfg, capacity=init["capacity"])
    dt = sim.dt
    lk = _antenna_laser(W, cfg.dz, row, P.beta, 0.5 * nst * dt)
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    sim.antenna(P.make_laser(**lk), row)
    sim.pic_step(nst)
    dg = sim.diagnostics(lineout=True)
    fg = {c: sim.get_field(c).cpu().numpy() for c in COMPS}
    sim.close()
    kw, oinit = resolve_oracle(W)
    s = O.Sim(**kw)
    s.set_threads(min(8, max(1, O.max_threads())))
    s.init(n_uniform=oinit["n_lab"], laser=oinit["laser"])
    s.set_antenna(O.make_laser(**lk), row)
    s.step(nst)
    do = s.diagnostics(lineout=True)
    for k in ("ue", "ub", "ukin"):
        assert abs(dg[k] - do[k]) <= 1e-5 * abs(do[k]), (k, dg[k], do[k])
    fo = {c: s.get_field(c) for c in COMPS}
    for c in COMPS:
        scale = np.abs(fo[c]).max()
        assert np.abs(fg[c] - fo[c]).max() <= 1e-5 * scale, c
    # the antenna did emit: without it the oracle's E_y differs from the
    # antenna run by more than half the target amplitude at the antenna
    s2 = O.Sim(**kw)
    s2.set_threads(min(8, max(1, O.max_threads())))
    s2.init(n_uniform=oinit["n_lab"], laser=oinit["laser"])
    s2.step(nst)
    las = O.make_laser(**lk)
    amp = max(abs(O.laser_eval(las, cfg.dim, W["gamma_b"], row * cfg.dz, 0.0, 0.0, t)[1])
              for t in np.linspace(0.0, nst * dt, 9))
    dey = np.abs(s2.get_field("Ey") - fo["Ey"]).max()
    print("antenna field", dey, "target amplitude", amp, flush=True)
    assert dey > 0.5 * amp


def test_antenna_emits_the_target_pulse_fp32(P):
    print("case antenna emission fp32", flush=True)
    gb, cells = 5.0, 32
    dz = P.boosted_dz(gb, LAMBDA0, cells)
    nz, dx = 32 * cells, 16 * LAMBDA0
    cfg = P.make_config(dim=2, nz=nz, nx=4, dz=dz, dx=dx, cfl=0.95, shape_order=1,
                        precision=P.FP32_SPLIT, z_boundary=P.BC_MUR, ppc=1)
    sim = P.Simulation(cfg, capacity=64)
    sim.init_boosted_plasma(gb)
    row = 40
    b = P.beta(gb)
    dop = 1.0 / (gb * (1.0 + b))
    L = 4 * LAMBDA0
    Lb = L / dop
    zc = row * dz - 4.5 * Lb
    lk = dict(a0=1.0, w0=0.0, L=L, z_center=dop * zc, z_focus=gb * zc, collimated=1)
    sim.antenna(P.make_laser(**lk), row)
    n = int((9.0 * Lb + 0.4 * (nz - row) * dz) / sim.dt)
    sim.pic_step(n)
    ey = sim.get_field("Ey").cpu().numpy()[:, 0, 0]
    sim.close()
    las = O.make_laser(**lk)
    i = np.arange(nz + 1)
    ana = np.array([O.laser_eval(las, 2, gb, k * dz, 0.0, 0.0, n * sim.dt)[1] for k in i])
    fw = i > row + 2
    err = np.linalg.norm(ey[fw] - ana[fw]) / np.linalg.norm(ana[fw])
    print("emitted pulse L2", err, flush=True)
    assert err < 0.05


def test_antenna_error_paths(P):
    W = WORKLOADS["adjoint_2d_tiny"]
    cfg, init, nst = resolve_gpu(W, precision="fp64", sort_interval=0)
    sim = P.Simulation(cfg, capacity=init["capacity"])
    las = P.make_laser(a0=1.0, L=10.0)
    with pytest.raises(P.BfpicError):
        sim.antenna(las, 10)  # before init
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    with pytest.raises(P.BfpicError):
        sim.antenna(las, 0)
    with pytest.raises(P.BfpicError):
        sim.antenna(las, cfg.nz)
    sim.antenna(las, 10)
    with pytest.raises(P.BfpicError):
        sim.forward_loss(nst, 10, nst - 5, nst, (10, 20, 4, 12))
    sim.antenna(None)
    sim.close()
