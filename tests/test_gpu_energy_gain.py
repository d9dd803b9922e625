"""GPU: energy gain of witness electrons in laser wakes at four lab densities
(the rescaled gain-versus-position curves of section "Modeling of up to 1 TeV
stages", Fig. 4), downscaled: n = 2e-3 .. 2.5e-4 n_c, gamma_b = gamma_g / 2
from 11 to 32 (recipe: ``workloads.gain_scaling``).

The gain of a stage scales as 1 / n and its length as the dephasing length
L_phi = lambda_p^3 / lambda0^2 (proportional to n^-3/2); the paper checks this
by rescaling every stage's curve to one.  Checked here:
  * the peak of n * gain, with gain the mean of gamma - gamma_0 over the 16
    most energetic witnesses (the leading slice of the bunch; the single most
    energetic witness rides on the plasma noise, up to 15% above), agrees
    across the densities within 8% of the mean;
  * the rescaled curves agree at z = L_phi within 8% of their mean (observed:
    0.85 to 0.90);
  * the gain peaks inside the run and falls after it (dephasing);
  * no NaN: the drifting plasma stays stable with c dt / dz' near 1 and the
    recipe's filtering.
The same stage (1e-3 n_c) run in two calculation frames, gamma_b = 0.5 and
0.85 gamma_g (box and run length by the same rules, 1550 and 750 steps), gives
the same lab-frame peak gain within 8%: the boosted frame changes the cost,
not the physics.
No oracle: the oracle would take minutes per density; the witness push it
checks is covered by the parity tests of the witness electrons.
"""
import math

import numpy as np
import pytest

from workloads import GAIN_DENSITIES, gain_scaling, resolve_gpu

pytestmark = pytest.mark.gpu

TOP = 16


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1011_0917_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def run_stage(P, n, every=10, ratio=0.5):
    import torch
    W = gain_scaling(n, ratio)
    wt = W["witness"]
    cfg, init, steps = resolve_gpu(W)
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    gb = init["gamma_b"]
    bb = P.beta(gb)
    gw = wt["gamma_lab"]
    S = np.zeros((wt["n"], 6))
    S[:, 0] = np.linspace(wt["z_centre"] - 1.6 * wt["wake_cells"],
                          wt["z_centre"] - 0.1 * wt["wake_cells"], wt["n"])
    S[:, 1] = np.linspace(0.0, W["nx"], wt["n"], endpoint=False)
    S[:, 3] = gb * (math.sqrt(gw * gw - 1.0) - bb * gw)
    Sg = torch.from_numpy(S).to(sim.device)
    sim.witness_bind(Sg)
    lab0 = sim.witness_lab().cpu().numpy()
    curve = []
    for _ in range(steps // every):
        sim.pic_step(every)
        lab = sim.witness_lab().cpu().numpy()
        live = Sg[:, 0].cpu().numpy() > 0.0
        gain = np.where(live, lab[:, 2] - lab0[:, 2], -np.inf)
        top = np.argsort(gain)[-TOP:]
        assert np.isfinite(gain[top]).all()
        dz = (lab[top, 1] - lab0[top, 1]).mean()
        curve.append((dz / wt["dephasing"], n * gain[top].mean(), n * gain[top[-1]]))
    d = sim.diagnostics()
    sim.close()
    return np.array(curve), d


def test_energy_gain_scales_as_inverse_density(P):
    peaks, at_lphi = [], []
    for n in GAIN_DENSITIES:
        print("case energy gain, n =", n, flush=True)
        c, d = run_stage(P, n)
        assert not d["nan_flag"]
        i = int(np.argmax(c[:, 1]))
        peaks.append(c[i, 1])
        # first crossing of z = L_phi on the (rising) rescaled curve
        k = int(np.argmax(c[:, 0] >= 1.0))
        assert c[k, 0] >= 1.0 and k > 0
        f = (1.0 - c[k - 1, 0]) / (c[k, 0] - c[k - 1, 0])
        at_lphi.append(c[k - 1, 1] + f * (c[k, 1] - c[k - 1, 1]))
        print(f"n={n:.2e} peak n*gain={c[i, 1]:.4f} at z/L_phi={c[i, 0]:.3f}, "
              f"n*gain at L_phi={at_lphi[-1]:.4f}, end {c[-1, 1]:.4f}, "
              f"best single witness {c[:, 2].max():.4f}", flush=True)
        assert c[-1, 1] < 0.97 * c[i, 1]  # past the peak: dephasing
    peaks, at_lphi = np.array(peaks), np.array(at_lphi)
    assert np.abs(peaks / peaks.mean() - 1.0).max() < 0.08
    assert np.abs(at_lphi / at_lphi.mean() - 1.0).max() < 0.08


def test_energy_gain_is_frame_independent(P):
    peaks = {}
    for ratio in (0.5, 0.85):
        print("case energy gain at 1e-3 n_c, gamma_b / gamma_g =", ratio, flush=True)
        c, d = run_stage(P, 1e-3, ratio=ratio)
        assert not d["nan_flag"]
        i = int(np.argmax(c[:, 1]))
        peaks[ratio] = c[i, 1]
        print(f"gamma_b / gamma_g = {ratio}: peak n*gain {c[i, 1]:.4f} at z/L_phi {c[i, 0]:.3f}",
              flush=True)
    assert abs(peaks[0.85] / peaks[0.5] - 1.0) < 0.08
