"""GPU: the FP32 split form against the FP64 form at the full sizes of the
gamma_b = 130 throughput run (8192 x 512, 8 ppc, 5000 steps) and of the 3D run
(gamma_b = 100, 512 x 128 x 128, quadratic shapes, 1000 steps).

The oracle cannot run these sizes; the FP64 form is the oracle's stand-in
here, pinned to it element by element on the smaller boxes of the same
physics.  Tolerances (for the FP32 form at these sizes): U_E, U_B within
1e-3 relative and the on-axis Ez lineout within 2e-2 (L2), checked at every
diagnostic sample up to and including the onset of the numerical
instability: the first sample at which the FP64 field energy U_E + U_B has
more than doubled over the preceding window (500 steps in 2D, 100 in 3D).
Past the onset the growth amplifies every difference between the two forms
(observed at the last step: 2.4e-3 on U_E in 2D, 2.5e-2 on U_B in 3D), and
the onset step is printed.
"""
import numpy as np
import pytest

from workloads import WORKLOADS, resolve_gpu

pytestmark = pytest.mark.gpu

CASES = {"boost130_2d": (250, 500), "boost100_3d": (50, 100)}


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1011_0917_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def history(P, name, precision, every):
    W = WORKLOADS[name]
    cfg, init, nst = resolve_gpu(W, precision=precision, sort_interval=50)
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    out = []
    for s in range(0, nst + 1, every):
        if s:
            sim.pic_step(every)
        d = sim.diagnostics(lineout=True)
        assert not d["nan_flag"]
        out.append((s, d["ue"], d["ub"], d["lineout"]))
    sim.close()
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_against_fp64_before_the_instability_onset(P, name):
    every, window = CASES[name]
    print("case", name, "fp32 and fp64 histories", flush=True)
    h32 = history(P, name, "fp32", every)
    h64 = history(P, name, "fp64", every)
    u = np.array([x[1] + x[2] for x in h64])
    back = window // every
    onset = None
    for k in range(back, len(u)):
        if u[k] > 2.0 * u[k - back]:
            onset = k
            break
    last = onset if onset is not None else len(u) - 1
    print(f"{name}: instability onset at step {h64[last][0] if onset is not None else None}; "
          f"U_E + U_B {u[0]:.3e} at step 0, {u[last]:.3e} at the onset, {u[-1]:.3e} at the end",
          flush=True)
    for k in range(last + 1):
        (s, ue, ub, lo), (_, ue64, ub64, lo64) = h32[k], h64[k]
        assert abs(ue - ue64) <= 1e-3 * ue64, (s, ue, ue64)
        assert abs(ub - ub64) <= 1e-3 * ub64, (s, ub, ub64)
        if np.linalg.norm(lo64) > 0:
            assert np.linalg.norm(lo - lo64) <= 2e-2 * np.linalg.norm(lo64), s
    (s, ue, ub, _), (_, ue64, ub64, _) = h32[-1], h64[-1]
    print(f"{name} at step {s}: U_E rel {abs(ue - ue64) / ue64:.2e}, "
          f"U_B rel {abs(ub - ub64) / ub64:.2e}", flush=True)
