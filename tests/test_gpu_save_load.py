"""GPU: checkpoint and resume (pic_save / pic_load).

In the deterministic mode the current sums do not depend on the order of
the particles, so a run saved at step N, restored into a fresh context (which
re-sorts its particles) and continued must reproduce the uninterrupted run
bitwise: every field component, the energies and the live count.  Checked in
2D with the moving window and continuous injection (the injection cursor and
the window schedule are part of the state), in 3D with quadratic shapes, and
through a copy of the blob to the host and back.  In the plain FP32 mode the
order of the atomic sums differs, so there the bar is the FP32 tolerance
(1e-4 on the energies).  Error paths: a short blob, a blob that is not a
state, a blob of another configuration, and a save before init.
"""
import numpy as np
import pytest

from workloads import WORKLOADS, resolve_gpu, small

pytestmark = pytest.mark.gpu

COMPS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1011_0917_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def _new(P, W, det):
    cfg, init, nst = resolve_gpu(W, precision="fp32", sort_interval=20)
    cfg.deterministic = det
    sim = P.Simulation(cfg, capacity=init["capacity"])
    return sim, init, nst


def _state(sim):
    d = sim.diagnostics()
    f = {c: sim.get_field(c).cpu().numpy() for c in COMPS}
    return d, f


@pytest.mark.parametrize("name,via_host", [("boost13_2d_small", False),
                                           ("boost13_2d_small", True),
                                           ("boost100_3d_small", False)])
def test_resume_is_bitwise_in_deterministic_mode(P, name, via_host):
    W = WORKLOADS[name]
    print("case save/load", name, "via host" if via_host else "", flush=True)
    a, init, nst = _new(P, W, 1)
    a.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    half = nst // 2 + 3
    a.pic_step(half)
    blob = a.save()
    if via_host:
        blob = blob.cpu().clone()
    a.pic_step(nst - half)
    da, fa = _state(a)
    a.close()
    b, _, _ = _new(P, W, 1)
    b.load(blob)
    assert b.diagnostics()["step"] == half
    b.pic_step(nst - half)
    db, fb = _state(b)
    b.close()
    assert da["step"] == db["step"] == nst
    assert da["window_cells"] == db["window_cells"]
    if name.startswith("boost13"):
        assert da["window_cells"] > 0  # the window moved across the save
    assert da["live"] == db["live"]
    for k in ("ue", "ub", "ukin"):
        assert da[k] == db[k], k
    for c in COMPS:
        assert np.array_equal(fa[c], fb[c]), c


def test_resume_in_fp32_within_tolerance(P):
    W = WORKLOADS["boost13_2d_small"]
    print("case save/load fp32 plain", flush=True)
    a, init, nst = _new(P, W, 0)
    a.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    a.pic_step(40)
    blob = a.save()
    a.pic_step(nst - 40)
    da, _ = _state(a)
    a.close()
    b, _, _ = _new(P, W, 0)
    b.load(blob)
    b.pic_step(nst - 40)
    db, _ = _state(b)
    b.close()
    assert da["live"] == db["live"]
    for k in ("ue", "ub", "ukin"):
        assert abs(da[k] - db[k]) <= 1e-4 * abs(da[k]), k


def test_save_load_error_paths(P):
    import ctypes as C
    import torch
    W = WORKLOADS["boost13_2d_small"]
    a, init, _ = _new(P, W, 1)
    L = P.lib()
    n = C.c_int64()
    assert L.bfpic_state_bytes(a.h, C.byref(n)) != 0                  # before init
    dummy = torch.zeros(8192, dtype=torch.uint8, device=a.device)
    assert L.pic_save(a.h, C.c_void_p(dummy.data_ptr()), 8192) != 0   # before init
    a.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    a.pic_step(3)
    assert L.pic_save(a.h, C.c_void_p(dummy.data_ptr()), 8192) != 0   # too small
    assert L.pic_load(a.h, C.c_void_p(dummy.data_ptr()), 8192) != 0   # not a state
    blob = a.save()
    assert L.pic_load(a.h, C.c_void_p(blob.data_ptr()), 1000) != 0    # shorter than the header says
    other, oinit, _ = _new(P, small("boost13_2d", nz=128, nx=64, ppc=4), 1)
    with pytest.raises(P.BfpicError):                                 # another configuration
        other.load(blob)
    other.close()
    with pytest.raises(P.BfpicError):                                 # not a uint8 blob
        a.load(blob.float())
    a.load(blob)                                                      # the round trip itself
    assert a.diagnostics()["step"] == 3
    a.close()
