"""GPU: the energy-conserving (Galerkin) gather against the oracle's.

* FP64 element by element against the FP64 oracle with the same gather form,
  at 1e-5 (the bar of every FP64 parity test): the lab run, the boosted 2D
  runs at gamma_b = 13 and 130, and the 3D quadratic run on both of its paths
  (the global-memory tiled path and the plain global path);
* the FP32 split form at the stated FP32 tolerances;
* witness electrons gathering in the Galerkin form from random vacuum fields,
  within 1e-11 of the oracle's FP64 push;
* the adjoint through the Galerkin gather against central differences, with
  quadratic shapes (the reduced shape is then linear and the loss stays
  continuous; with linear shapes the order-0 read jumps as a particle crosses
  a cell boundary, so differences of the loss straddle jumps).
"""
import numpy as np
import pytest

import oracle as O
from oracle import witness as WT
from workloads import WORKLOADS, adjoint_setup, resolve_gpu, resolve_oracle, small, witness_beam

pytestmark = pytest.mark.gpu

COMPS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1011_0917_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def _gpu(P, W, precision):
    cfg, init, nst = resolve_gpu(W, precision=precision)
    assert cfg.gather_form == P.GATHER_ENERGY
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    sim.pic_step(nst)
    d = sim.diagnostics(lineout=True)
    f = {c: sim.get_field(c).cpu().numpy() for c in COMPS}
    sim.close()
    return d, f


def _oracle(W):
    kw, init = resolve_oracle(W)
    assert kw["gather"] == 1
    s = O.Sim(**kw)
    s.set_threads(min(8, max(1, O.max_threads())))
    s.init(n_uniform=init["n_lab"], laser=init["laser"])
    s.step(W["steps"])
    return s.diagnostics(lineout=True), {c: s.get_field(c) for c in COMPS}


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


CASES = {"lab_2d": WORKLOADS["lab_2d"],
         "boost13_2d_small": WORKLOADS["boost13_2d_small"],
         "boost130_2d_small": WORKLOADS["boost130_2d_small"],
         "boost100_3d_small": WORKLOADS["boost100_3d_small"],
         "boost100_3d_tiled": WORKLOADS["boost100_3d_tiled"]}


@pytest.mark.parametrize("name", list(CASES))
def test_galerkin_fp64_matches_oracle(P, name):
    W = dict(CASES[name], gather="energy")
    print("case galerkin fp64", name, flush=True)
    dg, fg = _gpu(P, W, "fp64")
    do, fo = _oracle(W)
    for k in ("ue", "ub", "ukin"):
        assert _rel(dg[k], do[k]) < 1e-5, (k, dg[k], do[k])
    lo = np.linalg.norm(dg["lineout"] - do["lineout"]) / np.linalg.norm(do["lineout"])
    assert lo < 1e-5, lo
    assert dg["live"] == do["live"] and not dg["nan_flag"]
    for c in COMPS:
        scale = np.abs(fo[c]).max()
        assert np.abs(fg[c] - fo[c]).max() <= 1e-5 * scale, c


def test_galerkin_differs_from_momentum_form(P):
    """The two forms are different schemes: the fields after the same run differ."""
    W = dict(WORKLOADS["boost13_2d_small"], gather="energy")
    dg, _ = _gpu(P, W, "fp64")
    cfg, init, nst = resolve_gpu(WORKLOADS["boost13_2d_small"], precision="fp64")
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    sim.pic_step(nst)
    dm = sim.diagnostics()
    sim.close()
    assert _rel(dg["ue"], dm["ue"]) > 1e-6


@pytest.mark.parametrize("name", ["boost130_2d_small", "boost100_3d_small"])
def test_galerkin_fp32_split_within_tolerance(P, name):
    W = dict(CASES[name], gather="energy")
    print("case galerkin fp32", name, flush=True)
    dg, _ = _gpu(P, W, "fp32")
    do, _ = _oracle(W)
    assert _rel(dg["ue"], do["ue"]) < 1e-3
    assert _rel(dg["ub"], do["ub"]) < 1e-3
    lo = np.linalg.norm(dg["lineout"] - do["lineout"]) / np.linalg.norm(do["lineout"])
    assert lo < 2e-2, lo
    assert abs(dg["live"] - do["live"]) <= 1e-3 * do["live"]


@pytest.mark.parametrize("case", ["2d_linear_periodic", "3d_quadratic_open"])
def test_galerkin_witnesses_match_oracle(P, case):
    import torch
    name, over = {"2d_linear_periodic": ("lab_2d", {}),
                  "3d_quadratic_open": ("boost100_3d_small", {})}[case]
    W = small(name, gather="energy", **over)
    print("case galerkin witnesses", case, flush=True)
    cfg, init, _ = resolve_gpu(W, precision="fp64")
    sim = P.Simulation(cfg, capacity=64)
    sim.init_boosted_plasma(init["gamma_b"])
    kw, _ = resolve_oracle(W)
    s = O.Sim(**kw)
    s.init()
    rng = np.random.default_rng(8)
    periodic = W["zbc"] == "periodic"
    for c in COMPS:
        a = rng.uniform(-0.3, 0.3, s.shape)
        if periodic or c in ("Ez", "Bx", "By"):
            a[W["nz"]] = 0.0
        s.set_field(c, a)
        sim.set_field(c, torch.from_numpy(a).to(sim.device))
    Wo = witness_beam(W, 200, seed=9)
    Wo[:, 3:] = rng.uniform(-1.5, 1.5, (200, 3))
    Wg = torch.from_numpy(Wo).to(sim.device)
    sim.witness_bind(Wg)
    for _ in range(20):
        sim.pic_step(1)
        WT.push(s, Wo)
        w0 = s.diagnostics()["window_cells"]
        s.step(1)
        Wo[:, 0] -= s.diagnostics()["window_cells"] - w0
    got = Wg.cpu().numpy()
    sim.close()
    assert np.abs(got - Wo).max() < 1e-11 * max(1.0, np.abs(Wo).max())


def test_galerkin_adjoint_matches_differences(P):
    W = small("adjoint_2d_tiny", order=2, gather="energy")
    print("case galerkin adjoint, quadratic", flush=True)
    cfg, init, nst = resolve_gpu(W, precision="fp64", sort_interval=0)
    dt = P.yee_dt(2, cfg.dz, cfg.dx, 1.0, cfg.cfl)
    a = adjoint_setup(W, cfg.dz, P.beta, dt)

    def run(a0, kn, grad=False):
        sim = P.Simulation(cfg, capacity=init["capacity"])
        las = P.Laser()
        for f, _ in P.Laser._fields_:
            setattr(las, f, getattr(init["laser"], f))
        las.a0 = a0
        sim.init_boosted_plasma(init["gamma_b"], knots_z=a["knots_z"], knots_n=list(kn),
                                laser=las)
        L = sim.forward_loss(nst, a["interval"], a["window"][0], a["window"][1], a["box"])
        g = sim.adjoint(len(kn)) if grad else None
        sim.close()
        return L, g

    a0, kn = init["laser"].a0, np.array(a["knots_n"])
    L, (da0, dn) = run(a0, kn, grad=True)
    h = 1e-6
    fd_a0 = (run(a0 * (1 + h), kn)[0] - run(a0 * (1 - h), kn)[0]) / (2 * h * a0)
    assert abs(da0 - fd_a0) <= 1e-4 * abs(fd_a0), (da0, fd_a0)
    fd = []
    for m in range(len(kn)):
        kp, km = kn.copy(), kn.copy()
        kp[m] *= 1 + h
        km[m] *= 1 - h
        fd.append((run(a0, kp)[0] - run(a0, km)[0]) / (2 * h * kn[m]))
    scale = max(abs(v) for v in fd)
    for m in range(len(kn)):
        assert abs(dn[m] - fd[m]) <= 1e-4 * scale, (m, dn[m], fd[m])
