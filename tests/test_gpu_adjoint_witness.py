"""GPU adjoint with the witness-beam energy in the loss: L = (field loss) +
w * mean lab energy gamma_b (gamma' + beta_b u'_z) of witness electrons after
the last step, differentiated with respect to a0 and the density knots.

Checked against
  * central differences (h = 1e-6) of the GPU's own plain FP64 forward, at
    1e-4 (the kink argument of the field-loss tests: a witness crossing a cell
    boundary is one more kink of the piecewise-smooth loss);
  * the oracle's gradient: central differences of the FP64 oracle run with
    its witnesses pushed alongside (``oracle/witness.py``), at 1e-4;
  * the FP32 adjoint against FP64 differences at 1e-3;
and the witness term is shown to carry a good part of the gradient (the
gradient with w = 1 differs from that with w = 0 by more than 10% of it).
"""
import numpy as np
import pytest

import oracle as O
from oracle import witness as WT
from workloads import WORKLOADS, adjoint_setup, resolve_gpu, resolve_oracle

pytestmark = pytest.mark.gpu

H = 1e-6
NW = 32


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1011_0917_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def setup(P, name, precision):
    W = WORKLOADS[name]
    cfg, init, nst = resolve_gpu(W, precision=precision, sort_interval=0)
    dt = P.yee_dt(2, cfg.dz, cfg.dx, 1.0, cfg.cfl)
    a = adjoint_setup(W, cfg.dz, P.beta, dt)
    i0, i1, j0, j1 = a["box"]
    rng = np.random.default_rng(W["seed"] + 3)
    S = np.zeros((NW, 6))
    S[:, 0] = rng.uniform(i0 - 4, i1 + 4, NW)
    S[:, 1] = rng.uniform(j0, j1, NW)
    S[:, 3] = rng.uniform(0.5, 2.0, NW)
    S[:, 4] = rng.normal(0.0, 0.05, NW)
    return W, cfg, init, nst, a, S


def gpu_run(P, cfg, init, nst, a, S, a0, kn, ww, grad=False):
    import torch
    sim = P.Simulation(cfg, capacity=init["capacity"])
    las = P.Laser()
    for f, _ in P.Laser._fields_:
        setattr(las, f, getattr(init["laser"], f))
    las.a0 = a0
    sim.init_boosted_plasma(init["gamma_b"], knots_z=a["knots_z"], knots_n=list(kn), laser=las)
    Sg = torch.from_numpy(S.copy()).to(sim.device)
    sim.witness_bind(Sg)
    L = sim.forward_loss(nst, a["interval"], a["window"][0], a["window"][1], a["box"],
                         witness_weight=ww)
    out = (L, None, None)
    if grad:
        da0, dn = sim.adjoint(len(kn))
        out = (L, da0, np.array(dn))
    sim.close()
    return out


def fd(loss, a0, kn):
    """Central differences of loss(a0, kn): {-1: dL/da0, m: dL/dn_m}."""
    out = {-1: (loss(a0 * (1 + H), kn) - loss(a0 * (1 - H), kn)) / (2 * H * a0)}
    for m in range(len(kn)):
        kp, km = kn.copy(), kn.copy()
        kp[m] *= 1 + H
        km[m] *= 1 - H
        out[m] = (loss(a0, kp) - loss(a0, km)) / (2 * H * kn[m])
    return out


def compare(da0, dn, ref, tol):
    assert abs(da0 - ref[-1]) <= tol * abs(ref[-1]), (da0, ref[-1])
    scale = max(abs(ref[m]) for m in range(len(dn)))
    for m in range(len(dn)):
        assert abs(dn[m] - ref[m]) <= tol * scale, (m, dn[m], ref[m], scale)


@pytest.mark.parametrize("name", ["adjoint_2d_tiny", "adjoint_2d_small"])
def test_witness_energy_gradient_matches_differences_fp64(P, name):
    print("case", name, "fp64, witness energy in the loss", flush=True)
    W, cfg, init, nst, a, S = setup(P, name, "fp64")
    a0, kn = init["laser"].a0, np.array(a["knots_n"])
    L, da0, dn = gpu_run(P, cfg, init, nst, a, S, a0, kn, 1.0, grad=True)
    _, f0, n0 = gpu_run(P, cfg, init, nst, a, S, a0, kn, 0.0, grad=True)
    ref = fd(lambda x, k: gpu_run(P, cfg, init, nst, a, S, x, k, 1.0)[0], a0, kn)
    print("dL/da0 adjoint", da0, "differences", ref[-1], "without the witness term", f0,
          flush=True)
    compare(da0, dn, ref, 1e-4)
    g1 = np.concatenate([[da0], dn])
    g0 = np.concatenate([[f0], n0])
    assert np.abs(g1 - g0).max() > 0.1 * np.abs(g1).max()


def test_witness_energy_gradient_fp32_against_fp64_differences(P):
    print("case adjoint_2d_small fp32, witness energy in the loss", flush=True)
    W, cfg32, init, nst, a, S = setup(P, "adjoint_2d_small", "fp32")
    _, cfg64, _, _, _, _ = setup(P, "adjoint_2d_small", "fp64")
    a0, kn = init["laser"].a0, np.array(a["knots_n"])
    L, da0, dn = gpu_run(P, cfg32, init, nst, a, S, a0, kn, 1.0, grad=True)
    ref = fd(lambda x, k: gpu_run(P, cfg64, init, nst, a, S, x, k, 1.0)[0], a0, kn)
    compare(da0, dn, ref, 1e-3)


def oracle_loss(W, a, S0, a0, kn, ww):
    kw, init = resolve_oracle(W)
    s = O.Sim(**kw)
    las = init["laser"]
    las.a0 = a0
    s.init(knots_z=a["knots_z"], knots_n=list(kn), laser=las)
    i0, i1, j0, j1 = a["box"]
    w0, w1 = a["window"]
    S = S0.copy()
    acc = 0.0
    for n in range(1, W["steps"] + 1):
        WT.push(s, S)
        s.step(1)
        if w0 <= n <= w1:
            ez = np.asarray(s.get_field("Ez"))
            acc += float(ez[i0:i1 + 1, j0:j1 + 1].mean())
    d = s.diagnostics()
    lab = WT.lab(S, d["t"], d["window_cells"], kw["dz"], kw["gamma_b"])
    return acc / (w1 - w0 + 1) + ww * lab[:, 2].mean()


def test_witness_energy_gradient_matches_oracle(P):
    print("case adjoint_2d_tiny vs oracle differences, witness energy", flush=True)
    W, cfg, init, nst, a, S = setup(P, "adjoint_2d_tiny", "fp64")
    a0, kn = init["laser"].a0, np.array(a["knots_n"])
    L, da0, dn = gpu_run(P, cfg, init, nst, a, S, a0, kn, 1.0, grad=True)
    Lo = oracle_loss(W, a, S, a0, kn, 1.0)
    assert abs(L - Lo) <= 1e-10 * abs(Lo)
    ref = fd(lambda x, k: oracle_loss(W, a, S, x, k, 1.0), a0, kn)
    compare(da0, dn, ref, 1e-4)


def test_witness_rebinding_after_taped_run_is_refused(P):
    import torch
    W, cfg, init, nst, a, S = setup(P, "adjoint_2d_tiny", "fp64")
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], knots_z=a["knots_z"], knots_n=a["knots_n"],
                            laser=init["laser"])
    with pytest.raises(P.BfpicError):  # a witness weight without witnesses
        sim.forward_loss(4, 2, 1, 4, a["box"], witness_weight=1.0)
    Sg = torch.from_numpy(S.copy()).to(sim.device)
    sim.witness_bind(Sg)
    sim.forward_loss(4, 2, 1, 4, a["box"], witness_weight=1.0)
    sim.witness_bind(Sg[:8].contiguous())
    with pytest.raises(P.BfpicError):
        sim.adjoint(len(a["knots_n"]))
    sim.close()


def test_autograd_function_with_witnesses(P):
    import torch
    from paper_1011_0917_amd.adjoint import BoostedPICLoss, PICLossSpec
    print("case autograd function with witnesses", flush=True)
    W, cfg, init, nst, a, S = setup(P, "adjoint_2d_tiny", "fp64")
    laser = {f: getattr(init["laser"], f) for f, _ in P.Laser._fields_ if f != "a0"}
    spec = PICLossSpec(cfg=cfg, capacity=init["capacity"], gamma_boost=init["gamma_b"],
                       knots_z=a["knots_z"], laser=laser, nsteps=nst, interval=a["interval"],
                       step_first=a["window"][0], step_last=a["window"][1], box=a["box"],
                       witnesses=S, witness_weight=0.5)
    a0 = torch.tensor(init["laser"].a0, dtype=torch.float64, requires_grad=True)
    kn = torch.tensor(a["knots_n"], dtype=torch.float64, requires_grad=True)
    loss = BoostedPICLoss.apply(a0, kn, spec)
    loss.backward()
    L, da0, dn = gpu_run(P, cfg, init, nst, a, S, init["laser"].a0, np.array(a["knots_n"]),
                         0.5, grad=True)
    assert abs(float(loss) - L) <= 1e-12 * abs(L)
    assert abs(float(a0.grad) - da0) <= 1e-10 * abs(da0)
    assert np.allclose(kn.grad.numpy(), dn, rtol=1e-10, atol=1e-10 * np.abs(dn).max())


def test_witness_adjoint_3d_matches_differences(P):
    """3D (32 x 16 x 16): witnesses spread in y as well, the witness adjoint
    with the 3D gather transpose, FP64 against central differences at 1e-4."""
    print("case witness adjoint 3d", flush=True)
    W = WORKLOADS["adjoint_3d_tiny"]
    cfg, init, nst = resolve_gpu(W, precision="fp64", sort_interval=0)
    dt = P.yee_dt(3, cfg.dz, cfg.dx, cfg.dy, cfg.cfl)
    a = adjoint_setup(W, cfg.dz, P.beta, dt)
    i0, i1, j0, j1, k0, k1 = a["box"]
    rng = np.random.default_rng(W["seed"] + 5)
    S = np.zeros((NW, 6))
    S[:, 0] = rng.uniform(i0 - 4, i1 + 4, NW)
    S[:, 1] = rng.uniform(j0, j1, NW)
    S[:, 2] = rng.uniform(k0, k1, NW)
    S[:, 3] = rng.uniform(0.5, 2.0, NW)
    S[:, 4] = rng.normal(0.0, 0.05, NW)
    S[:, 5] = rng.normal(0.0, 0.05, NW)
    a0, kn = init["laser"].a0, np.array(a["knots_n"])
    L, da0, dn = gpu_run(P, cfg, init, nst, a, S, a0, kn, 1.0, grad=True)
    L0, da00, dn0 = gpu_run(P, cfg, init, nst, a, S, a0, kn, 0.0, grad=True)
    assert abs(da0 - da00) > 0.1 * abs(da0)  # the witness term carries the gradient
    g = fd(lambda x, k: gpu_run(P, cfg, init, nst, a, S, x, k, 1.0)[0], a0, kn)
    print("adjoint", da0, list(dn), "differences", g, flush=True)
    assert abs(da0 - g[-1]) <= 1e-4 * abs(g[-1])
    scale = max(abs(g[m]) for m in range(len(kn)))
    for m in range(len(kn)):
        assert abs(dn[m] - g[m]) <= 1e-4 * scale, (m, dn[m], g[m])
