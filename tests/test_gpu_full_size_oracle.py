"""GPU FP64 against the FP64 oracle at the full sizes of the three boosted
configurations, element by element, for a few steps:

* gamma_b = 13, 2048 x 256 cells, 8 ppc (4.2 M electrons), moving window;
* gamma_b = 130, 8192 x 512 cells, 8 ppc (33.5 M electrons);
* gamma_b = 100, 3D, 512 x 128 x 128 cells, 2 ppc (16.8 M electrons),
  quadratic shapes.

Each run takes one step, a forced re-sort of the GPU particles (which must
change nothing but the order of sums), then two more steps; the second step
injects the first new plasma column in 2D (its low edge enters as soon as
the plasma has drifted); in 3D the window moves backwards at the boosted
laser group velocity and shifts one cell back instead.  Tolerance (FP64 mode): 1e-5 relative on U_E, U_B,
U_kin and the on-axis Ez lineout (L2), every E and B node within 1e-5 of its
component's maximum, identical live counts, the same injected-column count.

The oracle runs on the host cores (OpenMP, per-thread current buffers).

Also: the FP32 split form against the FP64 form over the gamma_b = 13 run
at its full size, at the tolerances stated for it (U_E within 1e-3, the wake
Ez lineout within 1e-2 in L2) at every sample up to the onset of the
numerical instability, which this configuration reaches near step 550.
"""
import os

import numpy as np
import pytest

import oracle as O
from workloads import WORKLOADS, resolve_gpu, resolve_oracle

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))
COMPS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1011_0917_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _gpu(P, W):
    import torch
    cfg, init, _ = resolve_gpu(W, precision="fp64", sort_interval=0)
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    n0 = sim.num_slots()
    sim.pic_step(1)
    sim.sort()
    sim.pic_step(2)
    d = sim.diagnostics(lineout=True)
    f = {c: sim.get_field(c).cpu().numpy() for c in COMPS}
    n1 = sim.num_slots()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return d, f, n0, n1


def _oracle(W):
    kw, init = resolve_oracle(W)
    s = O.Sim(**kw)
    s.set_threads(THREADS)
    s.init(n_uniform=init["n_lab"], laser=init["laser"])
    n0 = s.num_pairs()
    s.step(3)
    d = s.diagnostics(lineout=True)
    f = {c: s.get_field(c) for c in COMPS}
    return d, f, n0


@pytest.mark.parametrize("name", ["boost13_2d", "boost130_2d", "boost100_3d"])
def test_full_size_fp64_matches_oracle(P, name):
    W = WORKLOADS[name]
    print(f"case {name} full size: gpu fp64", flush=True)
    dg, fg, g0, g1 = _gpu(P, W)
    print(f"case {name} full size: oracle on {THREADS} threads", flush=True)
    do, fo, o0 = _oracle(W)
    print(f"{name}: live {dg['live']} (gpu) {do['live']} (oracle), "
          f"U_E {dg['ue']:.12e} / {do['ue']:.12e}", flush=True)
    assert g0 == o0
    assert dg["live"] == do["live"] and g1 >= dg["live"]
    if W.get("window") != "group" or W["dim"] == 2:
        # a column was injected: the plasma drifts off its lattice at once
        assert do["live"] > o0
    else:
        # the 3D window moves backwards (the laser is slower than the frame):
        # it shifts one cell back after the first step, and no column is due
        assert dg["window_cells"] == -1.0
    for k in ("ue", "ub", "ukin"):
        assert _rel(dg[k], do[k]) < 1e-5, (k, dg[k], do[k])
    lo_g, lo_o = dg["lineout"], do["lineout"]
    assert np.linalg.norm(lo_g - lo_o) <= 1e-5 * np.linalg.norm(lo_o)
    assert dg["window_cells"] == do["window_cells"]
    assert not dg["nan_flag"]
    for c in COMPS:
        scale = np.abs(fo[c]).max()
        err = np.abs(fg[c] - fo[c]).max()
        print(f"  {c}: max |gpu - oracle| / max |oracle| = {err / max(scale, 1e-300):.2e}",
              flush=True)
        assert err <= 1e-5 * scale, c


def _history(P, W, precision, every, last):
    cfg, init, _ = resolve_gpu(W, precision=precision, sort_interval=50)
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    out = []
    for m in range(0, last + 1, every):
        if m:
            sim.pic_step(every)
        out.append((m, sim.diagnostics(lineout=True)))
    sim.close()
    return out


def test_boost13_full_run_fp32_against_fp64(P):
    """The gamma_b = 13 configuration as given (2048 x 256, dz' = 1.62 lambda0,
    dx = lambda0 / 4, c dt / dz' = 0.145, 4 passes with compensation) is
    numerically unstable: from step ~550 the drifting plasma's field energy
    grows by about 1e12 per 100 steps, in FP64 as in FP32, and FP32 overflows
    near step 1000 (the oracle shows the same growth on a smaller box of the
    same resolution).  The FP32 form is checked against the FP64 form at every
    sample up to and including the onset, which must not come before step
    500; the onset is the first sample at which the FP64 field energy has more
    than doubled over the preceding 500 steps (here step 500, where U_E + U_B
    is 2.9 times its value at step 0)."""
    W = WORKLOADS["boost13_2d"]
    every, last = 100, 800
    print("case boost13_2d full run: fp32 and fp64 histories", flush=True)
    h32 = _history(P, W, "fp32", every, last)
    h64 = _history(P, W, "fp64", every, last)
    u = np.array([d["ue"] + d["ub"] for _, d in h64])
    back = 500 // every
    onset = next((k for k in range(back, len(u)) if u[k] > 2.0 * u[k - back]), len(u))
    onset_step = h64[onset][0] if onset < len(u) else None
    print(f"boost13_2d: instability onset at step {onset_step}; U_E + U_B {u[0]:.3e} at "
          f"step 0, {u[min(onset, len(u) - 1)]:.3e} at the onset", flush=True)
    assert onset_step is not None and onset_step >= 500
    for k in range(len(u)):
        (m, a), (_, b) = h32[k], h64[k]
        e_ue = _rel(a["ue"], b["ue"])
        e_ub = _rel(a["ub"], b["ub"])
        e_lo = np.linalg.norm(a["lineout"] - b["lineout"]) / max(np.linalg.norm(b["lineout"]),
                                                                 1e-300)
        print(f"  step {m}: U_E rel {e_ue:.2e}, U_B rel {e_ub:.2e}, wake lineout L2 "
              f"{e_lo:.2e}, FP64 U_E {b['ue']:.4e}", flush=True)
        if k <= onset:
            assert not a["nan_flag"] and not b["nan_flag"]
            assert e_ue <= 1e-3 and e_ub <= 1e-3, (m, a["ue"], b["ue"], a["ub"], b["ub"])
            if m > 0:
                assert e_lo <= 1e-2, m
