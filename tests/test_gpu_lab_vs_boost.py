"""GPU: one stage in plasma simulated in the lab frame and in a frame boosted
at gamma = 5, compared in the lab frame (the comparison of the section
"Effect of the hyperbolic rotation in Minkowski space", Fig. 2: the on-axis
laser-field history of a lab run against the Lorentz-transformed history of
a boosted run, in the lab-frame window moving at the laser group velocity).

The stage (``workloads.lab_boost_pair``): a plane-wave pulse (a0 = 1,
resonant length L = sqrt(2) / k_p) enters a plasma of 0.01 n_c through a
linear ramp and drives a wake over 10 plasma wavelengths.  Both runs use the
same numerics (FP64, 4 binomial passes with compensation, linear shapes,
Mur ends, a window at the group velocity) at the same resolution of the
laser in their own frame.  The boosted run starts with the pulse in vacuum
on the whole t' = 0 hyperplane, so that its initial field is exact; the lab
run starts at the lab time the pulse is 150 c/omega0 from the plasma (vacuum
propagation being exact, the two describe the same stage).  Records: the
on-axis lab-frame E_y (``bfpic_axis_record``, frame 1) and the on-axis E_z
(invariant under the boost along z) of every step (boosted) or every second
step (lab), carried onto one lab (t, zeta = z - v_g t) grid by
``bfpic_back_transform``.

What fixes the tolerances:
* the laser history differs by the Yee phase error of each grid, which grows
  with the propagation time and falls as the square of the cell size: at 32
  cells per wavelength it is within 12% (L2) over the grid and 15% in the
  last tenth of it (observed 8% and 11%), and halving the cell divides the
  error of the last tenth by at least 3 (observed 4.1);
* the wake E_z agrees within 8% (L2; observed 3 to 6%) once the plasma front
  has left the compared window.  While the front crosses it, the boosted
  wake is up to 1.6 times the lab one, more so with more filtering in the
  boosted frame and least without: a transient of the drifting plasma's
  front, where the paper locates the numerical instability.
"""
import numpy as np
import pytest

from workloads import lab_boost_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1011_0917_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def _run(P, S, boosted):
    import torch
    R = S["boost"] if boosted else S["lab"]
    cfg = P.make_config(dim=2, nz=R["nz"], nx=S["nx"], dz=R["dz"], dx=S["dx"], cfl=S["cfl"],
                        shape_order=1, filter_passes=S["passes"], filter_compensate=1,
                        precision=P.FP64, z_boundary=P.BC_MUR, ppc=S["ppc"],
                        load=P.LOAD_CENTERED, sort_interval=20, seed=S["seed"],
                        beta_window=R["beta_window"], auto_window=1)
    sim = P.Simulation(cfg, capacity=R["nz"] * S["nx"] * S["ppc"] * 4)
    las = P.make_laser(a0=S["a0"], w0=0.0, L=S["L"], z_center=R["z_center"], z_focus=0.0,
                       collimated=1)
    sim.init_boosted_plasma(R["gamma_b"], knots_z=R["knots_z"], knots_n=R["knots_n"], laser=las)
    ey, ez, tp, z0 = [], [], [], []
    for n in range(R["steps"] + 1):
        if n:
            sim.pic_step(1)
        if n % R["every"]:
            continue
        r, m = sim.axis_record(1)
        d = sim.diagnostics(lineout=True)
        assert not d["nan_flag"]
        ey.append(r.cpu().numpy())
        ez.append(np.append(d["lineout"], 0.0))  # nz rows of Ez, padded to nz + 1
        tp.append(m["t_prime"])
        z0.append(m["z0_prime"])
    tp, z0 = np.array(tp), np.array(z0)
    out = {}
    # the original lab coordinates of the grid, in this run's coordinates
    g = S["grid"]
    t0 = g["t0"] - R["t_shift"]
    zeta0 = g["zeta0"] - R["z_shift"] + S["v_window"] * R["t_shift"]
    for name, rec, half in (("Ey", ey, 0.0), ("Ez", ez, 0.5)):
        out[name] = sim.back_transform(torch.tensor(np.array(rec)), tp, z0 + half * R["dz"],
                                       R["dz"], R["gamma_b"], t0, g["dt"], g["nt"], zeta0,
                                       g["dzeta"], g["nzeta"], S["v_window"]).cpu().numpy()
    sim.close()
    return out


def _l2(a, b, rows):
    f = np.isfinite(a[rows]) & np.isfinite(b[rows])
    assert f.sum() > 0.9 * f.size
    return np.linalg.norm(a[rows][f] - b[rows][f]) / np.linalg.norm(b[rows][f])


def _pair(P, cells):
    S = lab_boost_pair(P.beta, P.boosted_dz, P.boosted_group_beta, P.yee_dt, cells)
    print(f"case lab vs boost, {cells} cells per wavelength", flush=True)
    return S, _run(P, S, True), _run(P, S, False)


def test_boosted_stage_matches_lab_stage(P):
    S32, b32, l32 = _pair(P, 32)
    nt = S32["grid"]["nt"]
    allr, last = slice(0, nt), slice(nt - nt // 10, nt)
    e_all = _l2(b32["Ey"], l32["Ey"], allr)
    e_last32 = _l2(b32["Ey"], l32["Ey"], last)
    after = slice(S32["grid"]["front_gone"], nt)
    w_after = _l2(b32["Ez"], l32["Ez"], after)
    print(f"32 cells: laser L2 {e_all:.3f} (last tenth {e_last32:.3f}); wake after the front "
          f"{w_after:.3f}", flush=True)
    assert e_all < 0.12 and e_last32 < 0.15
    assert w_after < 0.08
    # the wake amplitude itself, against the lab run
    f = np.isfinite(b32["Ez"][after]) & np.isfinite(l32["Ez"][after])
    amp_b, amp_l = np.abs(b32["Ez"][after][f]).max(), np.abs(l32["Ez"][after][f]).max()
    assert abs(amp_b - amp_l) < 0.08 * amp_l
    S16, b16, l16 = _pair(P, 16)
    e_last16 = _l2(b16["Ey"], l16["Ey"], last)
    print(f"16 cells: laser L2 in the last tenth {e_last16:.3f}; ratio {e_last16 / e_last32:.2f}",
          flush=True)
    assert e_last16 > 3.0 * e_last32
