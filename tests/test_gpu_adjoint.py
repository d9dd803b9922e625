"""GPU adjoint: gradients of the Ez loss with respect to a0 and the density knots.

The reverse sweep (``pic_step_adjoint``) is checked against
  * central differences of the GPU's own FP64 forward (the discrete gradient
    the adjoint claims to be),
  * the oracle's gradient: central differences of the FP64 oracle run,
and the FP32 adjoint against FP64 differences, at the small, tiny and full
adjoint configurations.

The loss is a piecewise-smooth function of the parameters: with linear
shapes, the derivative jumps where a particle's path changes cells.  The
adjoint is the exact derivative at the operating point; a central difference
of step h straddles such a kink with a probability that grows with h and with
the number of particle-steps (at h = 1e-6 and ~5e5 particle-steps, about one
parameter in ten), and a straddled kink moves the quotient by ~1e-5 relative
(seen at h = 1e-4 on adjoint_2d_small: -1.5e-5, gone at h = 1e-6).  Hence
tolerances of 1e-4 against differences of step h = 1e-6, where FP64 round-off
in the quotient is ~1e-10 for a0.  The difference runs use the plain FP64
mode: its run-to-run noise (the order of the atomic sums) is ~1e-16 of the
loss, while the deterministic mode rounds every current contribution to 2^-40
of the largest one, which puts ~1e-4 of noise into a quotient at h = 1e-6.
The knot gradient is compared relative to its largest entry.
"""
import numpy as np
import pytest

import oracle as O
from workloads import WORKLOADS, adjoint_setup, resolve_gpu, resolve_oracle, small

pytestmark = pytest.mark.gpu

H = 1e-6


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
    return W, cfg, init, nst, a


def gpu_run(P, cfg, init, nst, a, a0, kn, grad=False, interval=None):
    sim = P.Simulation(cfg, capacity=init["capacity"])
    las = P.Laser()
    for f, _ in P.Laser._fields_:
        setattr(las, f, getattr(init["laser"], f))
    las.a0 = a0
    sim.init_boosted_plasma(init["gamma_b"], knots_z=a["knots_z"], knots_n=list(kn), laser=las)
    L = sim.forward_loss(nst, interval or a["interval"], a["window"][0], a["window"][1], a["box"])
    out = (L, None, None)
    if grad:
        da0, dn = sim.adjoint(len(kn))
        out = (L, da0, np.array(dn))
    sim.close()
    return out


def fd_gpu(P, cfg64, init, nst, a, which, h=H):
    """Central differences of the FP64 GPU loss for the parameters in `which`
    (-1: a0, m >= 0: knot m), in the plain FP64 mode (the least noisy one)."""
    cfg64.deterministic = 0
    a0, kn = init["laser"].a0, np.array(a["knots_n"])
    out = {}
    for m in which:
        if m < 0:
            lp = gpu_run(P, cfg64, init, nst, a, a0 * (1 + h), kn)[0]
            lm = gpu_run(P, cfg64, init, nst, a, a0 * (1 - h), kn)[0]
            out[m] = (lp - lm) / (2 * h * a0)
        else:
            kp, km = kn.copy(), kn.copy()
            kp[m] *= 1 + h
            km[m] *= 1 - h
            lp = gpu_run(P, cfg64, init, nst, a, a0, kp)[0]
            lm = gpu_run(P, cfg64, init, nst, a, a0, km)[0]
            out[m] = (lp - lm) / (2 * h * kn[m])
    return out


def compare(adj, fd, tol):
    """a0 relative to itself; the knot gradient relative to its largest entry
    (a small entry's difference quotient sits at the round-off floor: the loss
    moves by ~h n_m |dL/dn_m| / |L| relative)."""
    if -1 in fd:
        assert abs(adj[-1] - fd[-1]) <= tol * abs(fd[-1]), (-1, adj[-1], fd[-1])
    knots = [m for m in fd if m >= 0]
    if knots:
        scale = max(abs(fd[m]) for m in knots)
        for m in knots:
            assert abs(adj[m] - fd[m]) <= tol * scale, (m, adj[m], fd[m], scale)


def as_dict(da0, dn):
    d = {-1: da0}
    d.update({m: v for m, v in enumerate(dn)})
    return d


def test_adjoint_matches_differences_fp64(P):
    """No kink is straddled on this case at h = 1e-6: the observed agreement is
    ~1e-10 relative, so the tolerance is 1e-6."""
    print("case adjoint_2d_small fp64 vs differences", flush=True)
    W, cfg, init, nst, a = setup(P, "adjoint_2d_small", "fp64")
    L, da0, dn = gpu_run(P, cfg, init, nst, a, init["laser"].a0, a["knots_n"], grad=True)
    fd = fd_gpu(P, cfg, init, nst, a, [-1] + list(range(len(dn))))
    compare(as_dict(da0, dn), fd, 1e-6)


def test_adjoint_fp32_against_fp64_differences(P):
    print("case adjoint_2d_small fp32 adjoint vs fp64 differences", flush=True)
    W, cfg32, init, nst, a = setup(P, "adjoint_2d_small", "fp32")
    _, cfg64, _, _, _ = setup(P, "adjoint_2d_small", "fp64")
    L, da0, dn = gpu_run(P, cfg32, init, nst, a, init["laser"].a0, a["knots_n"], grad=True)
    fd = fd_gpu(P, cfg64, init, nst, a, [-1] + list(range(len(dn))))
    compare(as_dict(da0, dn), fd, 1e-4)


def test_adjoint_independent_of_checkpoint_interval(P):
    """Deterministic mode: the forward (and its recomputation from every
    checkpoint) repeats bitwise, so the loss is identical for every interval
    and the gradients agree to the order of the adjoint's own atomic sums."""
    print("case adjoint checkpoint interval", flush=True)
    W, cfg, init, nst, a = setup(P, "adjoint_2d_small", "fp64")
    cfg.deterministic = 1
    r1 = gpu_run(P, cfg, init, nst, a, init["laser"].a0, a["knots_n"], grad=True, interval=10)
    r2 = gpu_run(P, cfg, init, nst, a, init["laser"].a0, a["knots_n"], grad=True, interval=7)
    r3 = gpu_run(P, cfg, init, nst, a, init["laser"].a0, a["knots_n"], grad=True, interval=nst)
    for r in (r2, r3):
        assert r[0] == r1[0]
        assert abs(r[1] - r1[1]) <= 1e-10 * abs(r1[1])
        assert np.allclose(r[2], r1[2], rtol=1e-10, atol=1e-10 * np.abs(r1[2]).max())


def oracle_loss(W, a0, kn, a):
    kw, init = resolve_oracle(W)
    s = O.Sim(**kw)
    las = init["laser"]
    las.a0 = a0
    s.init(knots_z=a["knots_z"], knots_n=list(kn), laser=las)
    i0, i1, j0, j1, k0, k1 = tuple(a["box"]) + (0, 0) if len(a["box"]) == 4 else a["box"]
    w0, w1 = a["window"]
    acc = 0.0
    for n in range(1, W["steps"] + 1):
        s.step(1)
        if w0 <= n <= w1:
            ez = np.asarray(s.get_field("Ez"))
            acc += float(ez[i0:i1 + 1, j0:j1 + 1, k0:k1 + 1].mean())
    return acc / (w1 - w0 + 1)


def test_adjoint_matches_oracle_gradient(P):
    print("case adjoint_2d_tiny vs oracle differences", flush=True)
    W, cfg, init, nst, a = setup(P, "adjoint_2d_tiny", "fp64")
    L, da0, dn = gpu_run(P, cfg, init, nst, a, init["laser"].a0, a["knots_n"], grad=True)
    # the oracle's own loss agrees with the GPU loss
    a0, kn = init["laser"].a0, np.array(a["knots_n"])
    Lo = oracle_loss(W, a0, kn, a)
    assert abs(L - Lo) <= 1e-8 * abs(Lo)
    fd = {-1: (oracle_loss(W, a0 * (1 + H), kn, a) - oracle_loss(W, a0 * (1 - H), kn, a))
          / (2 * H * a0)}
    for m in range(len(kn)):
        kp, km = kn.copy(), kn.copy()
        kp[m] *= 1 + H
        km[m] *= 1 - H
        fd[m] = (oracle_loss(W, a0, kp, a) - oracle_loss(W, a0, km, a)) / (2 * H * kn[m])
    compare(as_dict(da0, dn), fd, 1e-4)


def test_autograd_function(P):
    import torch
    from paper_1011_0917_amd.adjoint import BoostedPICLoss, PICLossSpec
    print("case autograd function", flush=True)
    W, cfg, init, nst, a = setup(P, "adjoint_2d_small", "fp64")
    laser = {f: getattr(init["laser"], f) for f, _ in P.Laser._fields_ if f != "a0"}
    spec = PICLossSpec(cfg=cfg, capacity=init["capacity"], gamma_boost=init["gamma_b"],
                       knots_z=a["knots_z"], laser=laser, nsteps=nst, interval=a["interval"],
                       step_first=a["window"][0], step_last=a["window"][1], box=a["box"])
    a0 = torch.tensor(init["laser"].a0, dtype=torch.float64, requires_grad=True)
    kn = torch.tensor(a["knots_n"], dtype=torch.float64, requires_grad=True)
    loss = BoostedPICLoss.apply(a0, kn, spec)
    (2.0 * loss).backward()
    L, da0, dn = gpu_run(P, cfg, init, nst, a, init["laser"].a0, a["knots_n"], grad=True)
    assert abs(float(loss) - L) <= 1e-12 * abs(L)
    assert abs(float(a0.grad) - 2 * da0) <= 1e-10 * abs(da0)
    assert np.allclose(kn.grad.numpy(), 2 * dn, rtol=1e-10, atol=1e-10 * np.abs(dn).max())


def test_adjoint_full_config_fp32(P):
    """The adjoint configuration at full size (1024 x 128, 4 ppc, 500 steps,
    checkpoint every 50, 16 knots): the FP32 adjoint against FP64 differences
    on a0 and the three knots with the largest gradients."""
    print("case adjoint_2d full fp32", flush=True)
    W, cfg32, init, nst, a = setup(P, "adjoint_2d", "fp32")
    _, cfg64, _, _, _ = setup(P, "adjoint_2d", "fp64")
    L, da0, dn = gpu_run(P, cfg32, init, nst, a, init["laser"].a0, a["knots_n"], grad=True)
    top = list(np.argsort(-np.abs(dn))[:3])
    # at this size the many kinks average out; h = 1e-4 keeps the difference
    # well above round-off for the small knot gradients
    fd = fd_gpu(P, cfg64, init, nst, a, [-1] + [int(m) for m in top], h=1e-4)
    g = as_dict(da0, dn)
    print("loss", L, "adjoint", {m: g[m] for m in fd}, "differences", fd, flush=True)
    for m, v in fd.items():
        assert abs(g[m] - v) <= 1e-3 * abs(v), (m, g[m], v)


def _both_paths(P, W, precision):
    cfg, init, nst = resolve_gpu(W, precision=precision, sort_interval=0)
    cfg.deterministic = 1  # the taped forward repeats bitwise
    dt = P.yee_dt(2, cfg.dz, cfg.dx, 1.0, cfg.cfl)
    a = adjoint_setup(W, cfg.dz, P.beta, dt)
    out = []
    for per_direction in (True, False, False):
        sim = P.Simulation(cfg, capacity=init["capacity"])
        las = P.Laser()
        for f, _ in P.Laser._fields_:
            setattr(las, f, getattr(init["laser"], f))
        sim.init_boosted_plasma(init["gamma_b"], knots_z=a["knots_z"], knots_n=list(a["knots_n"]),
                                laser=las)
        L = sim.forward_loss(nst, a["interval"], a["window"][0], a["window"][1], a["box"])
        sim.adjoint_per_direction(per_direction)
        da0, dn = sim.adjoint(len(a["knots_n"]))
        sim.close()
        out.append((L, np.array([da0] + list(dn))))
    return out


@pytest.mark.parametrize("case", ["linear", "quadratic", "quadratic_galerkin"])
def test_staged_reverse_step_matches_per_direction(P, case):
    """The staged per-particle product (gather, push and deposit each evaluated
    once on a multi-tangent dual) against the twelve single-direction passes:
    the same gradient by the chain rule, FP64, to 1e-12 relative to the
    largest entry (observed: the order of the adjoint's atomic sums, which two
    runs of one path already differ by)."""
    W = {"linear": WORKLOADS["adjoint_2d_small"],
         "quadratic": small("adjoint_2d_tiny", order=2),
         "quadratic_galerkin": small("adjoint_2d_tiny", order=2, gather="energy")}[case]
    print("case staged adjoint", case, flush=True)
    (L1, g1), (L2, g2), (L3, g3) = _both_paths(P, W, "fp64")
    assert L1 == L2 == L3
    scale = np.abs(g1).max()
    print("per-direction vs staged", np.abs(g2 - g1).max() / scale,
          "staged run to run", np.abs(g3 - g2).max() / scale, flush=True)
    assert np.abs(g2 - g1).max() <= 1e-12 * scale
    assert np.abs(g3 - g2).max() <= 1e-12 * scale


def test_staged_reverse_step_fp32(P):
    print("case staged adjoint fp32", flush=True)
    (L1, g1), (L2, g2), _ = _both_paths(P, WORKLOADS["adjoint_2d_small"], "fp32")
    assert L1 == L2
    assert np.abs(g2 - g1).max() <= 1e-4 * np.abs(g1).max()


def _window_setup(P, precision):
    W = small("adjoint_2d_tiny", window="group")
    cfg, init, nst = resolve_gpu(W, precision=precision, sort_interval=0)
    assert cfg.auto_window == 1 and cfg.beta_window > 0.0
    dt = P.yee_dt(2, cfg.dz, cfg.dx, 1.0, cfg.cfl)
    a = adjoint_setup(W, cfg.dz, P.beta, dt, cfg.beta_window)
    return W, cfg, init, nst, a


def test_adjoint_with_moving_window_matches_differences(P):
    """The window at the boosted group velocity shifts 7 times over the 40
    taped steps; the reverse sweep applies each shift's transpose.  FP64
    adjoint against central differences of the FP64 forward (h = 1e-6,
    tolerance 1e-4 as for the kinked losses above), and the GPU's taped loss
    against the oracle's loss of the same windowed run."""
    print("case adjoint with moving window", flush=True)
    W, cfg, init, nst, a = _window_setup(P, "fp64")
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], knots_z=a["knots_z"], knots_n=a["knots_n"],
                            laser=init["laser"])
    sim.pic_step(nst)
    moved = sim.diagnostics()["window_cells"]
    sim.close()
    assert moved >= 5, moved
    L, da0, dn = gpu_run(P, cfg, init, nst, a, init["laser"].a0, a["knots_n"], grad=True)
    a0, kn = init["laser"].a0, np.array(a["knots_n"])
    Lo = oracle_loss(W, a0, kn, a)
    assert abs(L - Lo) <= 1e-8 * abs(Lo), (L, Lo)
    fd = fd_gpu(P, cfg, init, nst, a, [-1] + list(range(len(dn))))
    print("window cells", moved, "adjoint", da0, list(dn), "differences", fd, flush=True)
    compare(as_dict(da0, dn), fd, 1e-4)


def test_adjoint_with_moving_window_independent_of_checkpoint_interval(P):
    """Deterministic mode: restoring a checkpoint restores the window, so the
    loss is bitwise the same for every interval and the gradients agree."""
    print("case adjoint with moving window, checkpoint interval", flush=True)
    W, cfg, init, nst, a = _window_setup(P, "fp64")
    cfg.deterministic = 1
    r1 = gpu_run(P, cfg, init, nst, a, init["laser"].a0, a["knots_n"], grad=True, interval=10)
    r2 = gpu_run(P, cfg, init, nst, a, init["laser"].a0, a["knots_n"], grad=True, interval=7)
    assert r2[0] == r1[0]
    assert abs(r2[1] - r1[1]) <= 1e-10 * abs(r1[1])
    assert np.allclose(r2[2], r1[2], rtol=1e-10, atol=1e-10 * np.abs(r1[2]).max())


@pytest.mark.parametrize("order", [1, 2])
def test_adjoint_3d_matches_differences(P, order):
    """3D (32 x 16 x 16, linear and quadratic shapes): the reverse sweep with the
    3D Yee, Mur and filter transposes and the staged particle product over the
    3D deposit, FP64, against central differences of the FP64 forward (h = 1e-6,
    tolerance 1e-4), and the taped loss against the oracle's."""
    print("case adjoint 3d, order", order, flush=True)
    W = dict(WORKLOADS["adjoint_3d_tiny"], order=order)
    cfg, init, nst = resolve_gpu(W, precision="fp64", sort_interval=0)
    dt = P.yee_dt(3, cfg.dz, cfg.dx, cfg.dy, cfg.cfl)
    a = adjoint_setup(W, cfg.dz, P.beta, dt)
    assert len(a["box"]) == 6
    L, da0, dn = gpu_run(P, cfg, init, nst, a, init["laser"].a0, a["knots_n"], grad=True)
    a0, kn = init["laser"].a0, np.array(a["knots_n"])
    Lo = oracle_loss(W, a0, kn, a)
    assert abs(L - Lo) <= 1e-8 * abs(Lo), (L, Lo)
    fd = fd_gpu(P, cfg, init, nst, a, [-1] + list(range(len(dn))))
    print("adjoint", da0, list(dn), "differences", fd, flush=True)
    compare(as_dict(da0, dn), fd, 1e-4)


def test_adjoint_3d_fp32_against_fp64(P):
    print("case adjoint 3d fp32", flush=True)
    W = WORKLOADS["adjoint_3d_tiny"]
    res = {}
    for prec in ("fp64", "fp32"):
        cfg, init, nst = resolve_gpu(W, precision=prec, sort_interval=0)
        dt = P.yee_dt(3, cfg.dz, cfg.dx, cfg.dy, cfg.cfl)
        a = adjoint_setup(W, cfg.dz, P.beta, dt)
        res[prec] = gpu_run(P, cfg, init, nst, a, init["laser"].a0, a["knots_n"], grad=True)
    g64 = np.array([res["fp64"][1]] + list(res["fp64"][2]))
    g32 = np.array([res["fp32"][1]] + list(res["fp32"][2]))
    assert abs(g32[0] - g64[0]) <= 1e-3 * abs(g64[0])
    assert np.abs(g32[1:] - g64[1:]).max() <= 1e-3 * np.abs(g64[1:]).max()
