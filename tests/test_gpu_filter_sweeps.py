"""GPU: the 3D filter sweeps at the transverse sizes that select their forms.

The y sweep takes whole lines in one wave when ny is a multiple of 64 (one
register per 64 nodes, neighbours across lanes 0 and 63 from the adjacent
register) and windows of 64 - 2N nodes otherwise.  The full 512 x 128 x 128
box (two registers) is compared with the oracle elsewhere; here boosted 3D
runs (gamma_b = 100, quadratic shapes, 4 passes with compensation, tiled) at
ny = 64 and 192 (one and three registers) and ny = 40 (windows), FP64 against
the oracle: U_E, U_B, U_kin and the lineout at 1e-5, fields element by element
within 1e-5 of their maximum, identical live counts.
"""
import numpy as np
import pytest

import oracle as O
from workloads import resolve_gpu, resolve_oracle, small

pytestmark = pytest.mark.gpu

COMPS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1011_0917_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


@pytest.mark.parametrize("ny", [64, 192, 40])
def test_3d_sweeps_match_oracle(P, ny):
    W = small("boost100_3d", nz=32, nx=24, ny=ny, steps=10)
    print("case filter sweeps, ny =", ny, flush=True)
    cfg, init, nst = resolve_gpu(W, precision="fp64", sort_interval=5)
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    sim.pic_step(nst)
    dg = sim.diagnostics(lineout=True)
    fg = {c: sim.get_field(c).cpu().numpy() for c in COMPS}
    sim.close()
    kw, oinit = resolve_oracle(W)
    s = O.Sim(**kw)
    s.set_threads(min(16, max(1, O.max_threads())))
    s.init(n_uniform=oinit["n_lab"], laser=oinit["laser"])
    s.step(nst)
    do = s.diagnostics(lineout=True)
    for k in ("ue", "ub", "ukin"):
        assert abs(dg[k] - do[k]) <= 1e-5 * abs(do[k]), (k, dg[k], do[k])
    assert np.linalg.norm(dg["lineout"] - do["lineout"]) <= 1e-5 * np.linalg.norm(do["lineout"])
    assert dg["live"] == do["live"]
    for c in COMPS:
        fo = s.get_field(c)
        assert np.abs(fg[c] - fo).max() <= 1e-5 * np.abs(fo).max(), c
