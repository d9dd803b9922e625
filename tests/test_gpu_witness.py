"""GPU: witness electrons (test particles pushed in FP64 through the run's
fields) and their laboratory view, against the oracle (``oracle/witness.py``).

  * random fields in vacuum, both sides stepping the same FP64 Yee fields:
    witness state within 1e-11 after 20 steps (round-off), in open and
    periodic z, 2D and 3D, linear and quadratic shapes, across window shifts;
  * a full boosted run (plasma, laser, moving window) with a witness beam in
    the wake: a witness's momentum may drift from the oracle's by the gather
    error accumulated over the run, steps * dt * |F_gpu - F_oracle|max, with
    the field gap measured at the end of the same run; tested with a factor 4
    margin plus 1e-10 of round-off (observed: 6e-12 against a momentum change
    of 2);
  * closed form on the GPU alone: a uniform E_x turns u_x by -E_x dt per step;
  * the lab view against the oracle's to 1e-12 relative, and a witness at rest
    in the calculation frame seen at gamma_b, u_z = gamma_b beta_b.
"""
import numpy as np
import pytest

import oracle as O
from oracle import witness as WT
from workloads import WORKLOADS, resolve_gpu, resolve_oracle, small, witness_beam

pytestmark = pytest.mark.gpu

COMPS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")
HALF_Z = ("Ez", "Bx", "By")


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1011_0917_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def _pair(P, W, plasma):
    cfg, init, nst = resolve_gpu(W, precision="fp64")
    sim = P.Simulation(cfg, capacity=init["capacity"] if plasma else 64)
    kw, oinit = resolve_oracle(W)
    s = O.Sim(**kw)
    if plasma:
        sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
        s.init(n_uniform=oinit["n_lab"], laser=oinit["laser"])
    else:
        sim.init_boosted_plasma(init["gamma_b"])
        s.init()
    return sim, s


def _oracle_step(s, Wo):
    """One oracle step with the witnesses pushed through its start-of-step
    fields; positions follow the window."""
    WT.push(s, Wo)
    w0 = s.diagnostics()["window_cells"]
    s.step(1)
    Wo[:, 0] -= s.diagnostics()["window_cells"] - w0


VACUUM_CASES = {
    "2d_linear_periodic": ("lab_2d", {}),
    "2d_quadratic_open": ("boost13_2d_small", dict(order=2)),
    "3d_quadratic_open": ("boost100_3d_small", {}),
    "3d_linear_periodic": ("boost100_3d_small", dict(order=1, zbc="periodic", window=None)),
}


@pytest.mark.parametrize("case", list(VACUUM_CASES))
def test_witness_random_fields_match_oracle(P, case):
    import torch
    name, over = VACUUM_CASES[case]
    W = small(name, **over) if over else WORKLOADS[name]
    print("case witness vacuum", case, flush=True)
    sim, s = _pair(P, W, plasma=False)
    rng = np.random.default_rng(3)
    periodic = W["zbc"] == "periodic"
    for c in COMPS:
        a = rng.uniform(-0.3, 0.3, s.shape)
        if periodic or c in HALF_Z:
            a[W["nz"]] = 0.0
        s.set_field(c, a)
        sim.set_field(c, torch.from_numpy(a).to(sim.device))
    Wo = witness_beam(W, 200, seed=5)
    Wo[:, 3:] = rng.uniform(-1.5, 1.5, (200, 3))
    if periodic:  # witnesses across the z seam too
        Wo[:20, 0] = rng.uniform(0, 1, 20)
        Wo[20:40, 0] = W["nz"] - rng.uniform(0, 1, 20)
    Wg = torch.from_numpy(Wo).to(sim.device)
    sim.witness_bind(Wg)
    for n in range(20):
        if n == 10 and not periodic:
            sim.moving_window_shift(2)
            s.window_shift(2)
            Wo[:, 0] -= 2
        sim.pic_step(1)
        _oracle_step(s, Wo)
    got = Wg.cpu().numpy()
    sim.close()
    assert np.abs(got - Wo).max() < 1e-11 * max(1.0, np.abs(Wo).max())


def test_witness_beam_in_boosted_run_matches_oracle(P):
    import torch
    W = WORKLOADS["boost13_2d_small"]
    nst = W["steps"]
    print("case witness beam in boost13_2d_small fp64", flush=True)
    sim, s = _pair(P, W, plasma=True)
    Wo = witness_beam(W, 256)
    W0 = Wo.copy()
    Wg = torch.from_numpy(Wo).to(sim.device)
    sim.witness_bind(Wg)
    sim.pic_step(nst)
    for _ in range(nst):
        _oracle_step(s, Wo)
    got = Wg.cpu().numpy()
    lab_g = sim.witness_lab().cpu().numpy()
    d = sim.diagnostics()
    fgap = max(np.abs(sim.get_field(c).cpu().numpy() - s.get_field(c)).max() for c in COMPS)
    sim.close()
    du = np.abs(got[:, 3:] - Wo[:, 3:]).max()
    bound = 4 * nst * s.cfg.dt * fgap + 1e-10
    change = np.abs(Wo[:, 3:] - W0[:, 3:]).max()
    print("witness momentum gap", du, "bound", bound, "field gap", fgap, "momentum change",
          change, flush=True)
    assert du < bound
    assert change > 0.5  # the wake did act on the beam
    assert np.abs(got[:, :3] - Wo[:, :3]).max() < 1e-3
    lab_o = WT.lab(got, d["t"], d["window_cells"], s.cfg.dz, W["gamma_b"])
    assert np.abs(lab_g - lab_o).max() < 1e-12 * np.abs(lab_o).max()


def test_witness_uniform_field_closed_form(P):
    import torch
    W = WORKLOADS["lab_2d"]
    print("case witness uniform Ex", flush=True)
    cfg, init, _ = resolve_gpu(W)
    sim = P.Simulation(cfg, capacity=64)
    sim.init_boosted_plasma(init["gamma_b"])
    E0 = 0.21
    sim.set_field("Ex", torch.full(sim.field_shape, E0, dtype=torch.float64, device=sim.device))
    Wg = torch.tensor([[30.2, 10.7, 0.0, 0.4, 0.3, -0.2]], dtype=torch.float64,
                      device=sim.device)
    sim.witness_bind(Wg)
    sim.pic_step(25)
    got = Wg.cpu().numpy()[0]
    sim.close()
    assert abs(got[4] - (0.3 - 25 * sim.dt * E0)) < 1e-12
    assert got[3] == 0.4 and got[5] == -0.2


def test_witness_at_rest_lab_view(P):
    import torch
    W = WORKLOADS["boost13_2d_small"]
    cfg, init, _ = resolve_gpu(W, precision="fp64")
    sim = P.Simulation(cfg, capacity=64)
    sim.init_boosted_plasma(init["gamma_b"])
    Wg = torch.zeros((3, 6), dtype=torch.float64, device=sim.device)
    Wg[:, 0] = torch.tensor([10.0, 20.0, 30.0])
    sim.witness_bind(Wg)
    out = sim.witness_lab().cpu().numpy()
    sim.close()
    g = init["gamma_b"]
    b = P.beta(g)
    assert np.allclose(out[:, 2], g, rtol=1e-14) and np.allclose(out[:, 3], g * b, rtol=1e-14)
    # t' = 0: lab event (gamma_b beta_b z', gamma_b z')
    zp = np.array([10.0, 20.0, 30.0]) * cfg.dz
    assert np.allclose(out[:, 0], g * b * zp, rtol=1e-14)
    assert np.allclose(out[:, 1], g * zp, rtol=1e-14)


def test_witness_error_paths(P):
    import ctypes as C
    import torch
    W = WORKLOADS["adjoint_2d_tiny"]
    cfg, init, _ = resolve_gpu(W)
    sim = P.Simulation(cfg, capacity=init["capacity"])
    L = P.lib()
    dummy = C.c_void_p(1)
    assert L.bfpic_witness_bind(sim.h, 1, dummy) != 0        # before init
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    assert L.bfpic_witness_bind(sim.h, -1, dummy) != 0       # negative count
    assert L.bfpic_witness_bind(sim.h, 2, None) != 0         # null state
    assert L.bfpic_witness_lab(sim.h, dummy) != 0            # none bound
    with pytest.raises(P.BfpicError):
        sim.witness_bind(torch.zeros((4, 5), dtype=torch.float64, device=sim.device))
    Wg = torch.zeros((2, 6), dtype=torch.float64, device=sim.device)
    Wg[:, 0] = 20.0
    sim.witness_bind(Wg)
    with pytest.raises(P.BfpicError):                         # a weight that is not finite
        sim.forward_loss(2, 1, 1, 2, (0, 4, 0, 4), witness_weight=float("nan"))
    sim.witness_bind(None)
    assert L.bfpic_witness_lab(sim.h, dummy) != 0
    sim.close()
