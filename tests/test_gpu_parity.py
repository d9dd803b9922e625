"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances
  FP64 mode: 1e-5 relative on U_E, U_B, U_kin and on the on-axis Ez lineout (L2),
             field arrays element by element within 1e-5 of their maximum,
             identical live counts.
  FP32 split mode: the FP32 arithmetic of the push, deposit and field update
             against the FP64 oracle -- 1e-4 on U_E and U_kin in the lab frame,
             1e-3 on U_E and 1e-2 (L2) on the wake lineout in boosted frames.
  Sort: bit-exact permutation against the oracle's stable sort by (key, id).
"""
import math

import numpy as np
import pytest

import oracle as O
from workloads import WORKLOADS, resolve_gpu, resolve_oracle, small

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1011_0917_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def run_gpu(P, W, steps=None, precision=None, sort_interval=20, fields=True, det=0):
    cfg, init, nst = resolve_gpu(W, precision=precision, sort_interval=sort_interval)
    cfg.deterministic = det
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    sim.pic_step(nst if steps is None else steps)
    d = sim.diagnostics(lineout=True)
    f = {c: sim.get_field(c).cpu().numpy() for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")} \
        if fields else None
    sim.close()
    return d, f


def run_oracle(W, steps=None):
    kw, init = resolve_oracle(W)
    s = O.Sim(**kw)
    s.init(n_uniform=init["n_lab"], laser=init["laser"])
    s.step(W["steps"] if steps is None else steps)
    d = s.diagnostics(lineout=True)
    f = {c: s.get_field(c) for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")}
    return d, f


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def l2rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def check_fp64(dg, fg, do, fo, tol=1e-5):
    for k in ("ue", "ub", "ukin"):
        assert rel(dg[k], do[k]) < tol, (k, dg[k], do[k])
    assert l2rel(dg["lineout"], do["lineout"]) < tol
    assert dg["live"] == do["live"]
    assert not dg["nan_flag"]
    for c in fo:
        scale = max(np.abs(fo[c]).max(), 1e-300)
        assert np.abs(fg[c] - fo[c]).max() < tol * scale, c


# --------------------------------------------------------------------------
# Full-size lab configuration (128 x 64, 4 ppc, 200 steps), FP64
# --------------------------------------------------------------------------
def test_lab_2d_fp64_matches_oracle(P):
    W = WORKLOADS["lab_2d"]
    print("case lab_2d fp64", flush=True)
    dg, fg = run_gpu(P, W)
    do, fo = run_oracle(W)
    check_fp64(dg, fg, do, fo)
    # Gauss's law holds to round-off on the GPU too (periodic box)
    assert dg["gauss_res"] < 1e-12


def test_lab_2d_fp32_within_tolerance(P):
    W = WORKLOADS["lab_2d"]
    print("case lab_2d fp32", flush=True)
    dg, _ = run_gpu(P, W, precision="fp32", fields=False)
    do, _ = run_oracle(W)
    assert rel(dg["ue"], do["ue"]) < 1e-4
    assert rel(dg["ukin"], do["ukin"]) < 1e-4
    assert l2rel(dg["lineout"], do["lineout"]) < 1e-3
    assert dg["live"] == do["live"]


# --------------------------------------------------------------------------
# Boosted frames on small boxes: drift, injection, removal, window, Mur, filter
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["boost13_2d_small", "boost130_2d_small"])
def test_boosted_2d_fp64_matches_oracle(P, name):
    W = WORKLOADS[name]
    print("case", name, "fp64", flush=True)
    dg, fg = run_gpu(P, W, precision="fp64")
    do, fo = run_oracle(W)
    check_fp64(dg, fg, do, fo)
    assert dg["window_cells"] == do["window_cells"]


@pytest.mark.parametrize("name", ["boost13_2d_small", "boost130_2d_small"])
def test_boosted_2d_fp32_split_within_tolerance(P, name):
    W = WORKLOADS[name]
    print("case", name, "fp32", flush=True)
    dg, _ = run_gpu(P, W, precision="fp32", fields=False)
    do, _ = run_oracle(W)
    assert rel(dg["ue"], do["ue"]) < 1e-3
    assert rel(dg["ub"], do["ub"]) < 1e-3
    assert rel(dg["ukin_drift"], do["ukin_drift"]) < 1e-2
    assert l2rel(dg["lineout"], do["lineout"]) < 1e-2
    assert abs(dg["live"] - do["live"]) <= 1e-3 * do["live"]


@pytest.mark.parametrize("name", ["boost100_3d_small", "boost100_3d_tiled"])
def test_boosted_3d_fp64_matches_oracle(P, name):
    W = WORKLOADS[name]
    print("case", name, "fp64", flush=True)
    dg, fg = run_gpu(P, W, precision="fp64")
    do, fo = run_oracle(W)
    check_fp64(dg, fg, do, fo)


@pytest.mark.parametrize("name", ["boost100_3d_small", "boost100_3d_tiled"])
def test_boosted_3d_fp32_split_within_tolerance(P, name):
    W = WORKLOADS[name]
    print("case", name, "fp32", flush=True)
    dg, _ = run_gpu(P, W, precision="fp32", fields=False)
    do, _ = run_oracle(W)
    assert rel(dg["ue"] + dg["ub"], do["ue"] + do["ub"]) < 1e-3
    assert abs(dg["live"] - do["live"]) <= 1e-3 * do["live"]


# --------------------------------------------------------------------------
# Pairs pulled apart: electrons born with u_x = 10 (0.57 cells per step) drift
# about 15 cells across the 64-cell box in 100 steps, past their tile between
# sorts (stragglers) and away from their partners, whose current then leaves
# the tile's region (the far-partner deposit to the overflow grid).
# --------------------------------------------------------------------------
def test_separated_pairs_fp64_match_oracle(P):
    W = WORKLOADS["boost13_2d_small"]
    du = (10.0, 0.0, 0.0)
    print("case boost13_2d_small fp64 du_x = 10", flush=True)
    cfg, init, nst = resolve_gpu(W, precision="fp64", sort_interval=20)
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"], du=du)
    sim.pic_step(nst)
    dg = sim.diagnostics(lineout=True)
    fg = {c: sim.get_field(c).cpu().numpy() for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")}
    parts = sim.particles()
    sim.close()
    kw, oinit = resolve_oracle(W)
    s = O.Sim(**kw)
    s.init(n_uniform=oinit["n_lab"], laser=oinit["laser"], du=du)
    s.step(nst)
    do = s.diagnostics(lineout=True)
    fo = {c: s.get_field(c) for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")}
    check_fp64(dg, fg, do, fo)
    # the pairs really are apart: electron x against the partner's birth x
    live = parts["id"] >= 0
    ids = parts["id"][live].astype(np.int64)
    nx, ppc = W["nx"], W["ppc"]
    j = (ids // ppc) % nx
    k = ids // (ppc * nx)
    xs = np.array([j_ + O.cell_offset(W["seed"], k_, 0, j_, s_, 1, nx, 1, ppc)
                   for j_, k_, s_ in zip(j, k, ids % ppc)])
    sep = np.abs((parts["x"][live] - xs + nx / 2) % nx - nx / 2)
    print("median separation (cells)", float(np.median(sep)), flush=True)
    assert np.mean(sep > 6.0) > 0.5


# --------------------------------------------------------------------------
# Deterministic mode: int64 fixed-point current sums
# --------------------------------------------------------------------------
def _state(P, W, precision, det, steps):
    cfg, init, _ = resolve_gpu(W, precision=precision, sort_interval=20)
    cfg.deterministic = det
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    sim.pic_step(steps)
    f = {c: sim.get_field(c).cpu().numpy() for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz",
                                                      "Jx", "Jy", "Jz")}
    parts = sim.particles()
    d = sim.diagnostics(lineout=True)
    sim.close()
    return f, parts, d


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_deterministic_mode_repeats_bitwise(P, precision):
    W = WORKLOADS["boost13_2d_small"]
    print("case deterministic repeat", precision, flush=True)
    f1, p1, _ = _state(P, W, precision, 1, 60)
    f2, p2, _ = _state(P, W, precision, 1, 60)
    for c in f1:
        assert np.array_equal(f1[c], f2[c]), c
    for k in p1:
        assert np.array_equal(p1[k], p2[k]), k


def test_deterministic_mode_fp64_matches_oracle(P):
    for name in ("lab_2d", "boost13_2d_small"):
        W = WORKLOADS[name]
        print("case deterministic fp64", name, flush=True)
        dg, fg = run_gpu(P, W, precision="fp64", det=1)
        do, fo = run_oracle(W)
        check_fp64(dg, fg, do, fo)


def test_deterministic_mode_fp32_within_tolerance(P):
    W = WORKLOADS["boost130_2d_small"]
    print("case deterministic fp32 boost130_2d_small", flush=True)
    dg, _ = run_gpu(P, W, precision="fp32", fields=False, det=1)
    do, _ = run_oracle(W)
    assert rel(dg["ue"], do["ue"]) < 1e-3
    assert l2rel(dg["lineout"], do["lineout"]) < 1e-2


# --------------------------------------------------------------------------
# Sort: bit-exact against the oracle's stable sort by (key, id), interleaved
# inside each tile by rank within cell
# --------------------------------------------------------------------------
def interleave_tiles(perm, key, cpt):
    """Reorder a (key, id)-sorted permutation inside each tile of cpt cells by
    (rank within cell, cell), the layout the tiled particle kernel reads."""
    if cpt > 512:
        return perm
    k = key[perm]
    first = np.searchsorted(k, k, side="left")
    rank = np.arange(len(k)) - first
    return perm[np.lexsort((k % cpt, rank, k // cpt))]


@pytest.mark.parametrize("name,steps", [("boost13_2d_small", 0), ("boost13_2d_small", 37),
                                        ("lab_2d", 50), ("boost100_3d_small", 9)])
def test_sort_bit_exact(P, name, steps):
    W = WORKLOADS[name]
    print("case sort", name, steps, flush=True)
    cfg, init, _ = resolve_gpu(W, precision="fp64", sort_interval=0)
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    if steps:
        sim.pic_step(steps)
        sim.sort()
    s = sim.last_sort()
    keep = s["id"] >= 0
    perm = O.sort_perm(s["key"], s["id"])[: keep.sum()]
    tz, tx, ty = sim.tile_shape()
    assert np.array_equal(s["perm"], interleave_tiles(perm, s["key"], tz * tx * ty))
    if steps == 0:
        # identical initial states: the oracle computes the same keys itself
        kw, oi = resolve_oracle(W)
        o = O.Sim(**kw)
        o.init(n_uniform=oi["n_lab"], laser=oi["laser"])
        tz, tx, ty = sim.tile_shape()
        okey, oid = o.sort_keys(tz, tx, ty, s["tz_min"], s["ntz"])
        order = np.argsort(s["id"])
        oorder = np.argsort(oid)
        assert np.array_equal(s["id"][order], oid[oorder])
        assert np.array_equal(s["key"][order], okey[oorder])
    sim.close()


# --------------------------------------------------------------------------
# Yee dispersion on the GPU (no particles): exact discrete eigenmode
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_gpu_yee_dispersion(P, prec, tol):
    nz, nx, dz, dx = 64, 32, 0.7, 0.5
    cfg = P.make_config(dim=2, nz=nz, nx=nx, dz=dz, dx=dx, cfl=0.95,
                        precision=P.FP64 if prec == "fp64" else P.FP32_SPLIT)
    dt = P.yee_dt(2, dz, dx, 1.0, 0.95)
    sim = P.Simulation(cfg, capacity=16)
    sim.init_boosted_plasma(1.0)
    kz, kx = 2 * np.pi * 3 / (nz * dz), 2 * np.pi * 2 / (nx * dx)
    Kz, Kx = 2 * np.sin(kz * dz / 2) / dz, 2 * np.sin(kx * dx / 2) / dx
    K = math.hypot(Kz, Kx)
    w = 2 / dt * math.asin(K * dt / 2)
    i, j = np.meshgrid(np.arange(nz + 1), np.arange(nx), indexing="ij")

    def mode(n):
        c = math.cos(w * dt / 2)
        ey = np.cos(kz * i * dz + kx * j * dx - w * n * dt)
        bx = -Kz / K * c * np.cos(kz * (i + .5) * dz + kx * j * dx - w * n * dt)
        bz = Kx / K * c * np.cos(kz * i * dz + kx * (j + .5) * dx - w * n * dt)
        for a in (ey, bx, bz):
            a[nz] = 0
        return ey[..., None], bx[..., None], bz[..., None]

    ey, bx, bz = mode(0)
    sim.set_field("Ey", ey)
    sim.set_field("Bx", bx)
    sim.set_field("Bz", bz)
    sim.pic_step(80)
    ey, bx, bz = mode(80)
    for c, ref in (("Ey", ey), ("Bx", bx), ("Bz", bz)):
        got = sim.get_field(c).cpu().numpy()
        assert np.abs(got[:nz] - ref[:nz]).max() < tol, c
    sim.close()


# --------------------------------------------------------------------------
# Precision form: drifting cold plasma (k = 0 mode), closed form
# --------------------------------------------------------------------------
@pytest.mark.parametrize("gamma_b,prec,du,tol", [
    (13.0, "fp64", 1e-7, 1e-6), (130.0, "fp64", 1e-6, 1e-5),
    (13.0, "fp32", 3e-5, 1e-4), (130.0, "fp32", 3e-5, 1e-4), (1300.0, "fp32", 3e-5, 1e-4)])
def test_gpu_drifting_cold_plasma(P, gamma_b, prec, du, tol):
    """k = 0 mode of a cold plasma drifting at -beta_b (the precision-form gate).
    The linearised leapfrog gives E^n = E^1 sin(n th) / sin(th) with
    cos th = 1 - (n_lab / gamma_b^2) dt^2 / 2 (omega' = omega_p / gamma_b) and
    E^1 = dt n' dv, dv = v(u_b + du) - v(u_b) evaluated with 50 digits."""
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    nz, nx, dz, dx, n_lab = 16, 8, 1.0, 1.0, 0.1
    cfg = P.make_config(dim=2, nz=nz, nx=nx, dz=dz, dx=dx, cfl=0.95, ppc=1,
                        load=P.LOAD_CENTERED, sort_interval=0,
                        precision=P.FP64 if prec == "fp64" else P.FP32_SPLIT)
    dt = P.yee_dt(2, dz, dx, 1.0, 0.95)
    dU = du * gamma_b
    sim = P.Simulation(cfg, capacity=nz * nx)
    sim.init_boosted_plasma(gamma_b, n_uniform=n_lab, du=(0.0, 0.0, dU))
    g = Decimal(gamma_b)
    ub = -(g * g - 1).sqrt()
    v = lambda u: u / (1 + u * u).sqrt()
    dv = float(v(ub + Decimal(dU)) - v(ub))
    E1 = dt * gamma_b * n_lab * dv
    th = math.acos(1 - n_lab / gamma_b ** 2 * dt * dt / 2)
    nsteps = int(1.2 * math.pi / th)
    every = max(1, nsteps // 40)
    got, ns, n = [], [], 0
    while n + every <= nsteps:
        sim.pic_step(every)
        n += every
        got.append(sim.get_field("Ez").cpu().numpy()[:nz].mean())
        ns.append(n)
    got, ns = np.array(got), np.array(ns)
    pred = E1 * np.sin(ns * th) / math.sin(th)
    err = np.max(np.abs(got - pred)) / np.max(np.abs(pred))
    print("max rel err", err)
    assert err < tol
    sim.close()


# --------------------------------------------------------------------------
# Full size: the throughput configuration, sampled particles against the oracle
# --------------------------------------------------------------------------
def test_full_size_boost130_sampled_push(P):
    """At 8192 x 512 x 8 ppc (the benchmarked launch configuration), one more
    step of a random sample of particles matches the oracle's gather + Boris +
    move applied to the GPU's own fields and particle state."""
    import torch
    W = WORKLOADS["boost130_2d"]
    print("case full-size boost130 sampled", flush=True)
    cfg, init, _ = resolve_gpu(W)
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    sim.pic_step(5)
    d = sim.diagnostics()
    assert not d["nan_flag"] and d["live"] >= 8192 * 512 * 8
    f = {c: sim.get_field(c).cpu().numpy() for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")}
    p0 = sim.particles()
    live = np.nonzero(p0["id"] >= 0)[0]
    rng = np.random.default_rng(7)
    pick = rng.choice(live, 3000, replace=False)
    sim.pic_step(1)
    p1 = sim.particles()
    by_id = {int(i): k for k, i in enumerate(p1["id"])}
    kw, _ = resolve_oracle(W)
    kw = dict(kw, auto_window=0)
    o = O.Sim(**kw)
    o.init()  # vacuum, no plasma: only the sampled test electrons (w = 0)
    for c, a in f.items():
        o.set_field(c, a)
    for q in pick:
        o.add_pair(p0["z"][q], p0["x"][q], 0.0, p0["uz"][q], p0["ux"][q], p0["uy"][q],
                   p0["z"][q], p0["x"][q], 0.0, 0.0, int(p0["id"][q]))
    o.step(1)
    op = o.particles()
    ub = P.drift_u(W["gamma_b"])
    err = []
    for k, pid in enumerate(op["id"]):
        m = by_id[int(pid)]
        # peculiar momentum u - u_b z (FP32 state), and the new position (cells)
        for a, b in ((p1["ux"][m], op["ux"][k]), (p1["uy"][m], op["uy"][k]),
                     (p1["uz"][m] - ub, op["uz"][k] - ub)):
            err.append(abs(a - b) / (abs(b) + 1e-6))
        assert abs(p1["x"][m] - op["xe"][k]) < 1e-4
        assert abs(p1["z"][m] - op["ze"][k]) < 1e-4
    assert np.median(err) < 1e-5 and np.max(err) < 1e-2
    sim.close()


# --------------------------------------------------------------------------
# Error paths through the ABI
# --------------------------------------------------------------------------
def test_error_paths(P):
    W = small("boost13_2d", nz=64, nx=64, ppc=2)
    cfg, init, _ = resolve_gpu(W)
    sim = P.Simulation(cfg, capacity=100)
    with pytest.raises(P.BfpicError, match="ERR_STATE"):
        sim.pic_step(1)
    with pytest.raises(P.BfpicError, match="ERR_CAPACITY"):
        sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"])
    sim.close()
    cfgp = P.make_config(dim=2, nz=16, nx=8)
    sp = P.Simulation(cfgp, capacity=16)
    sp.init_boosted_plasma(1.0)
    with pytest.raises(P.BfpicError, match="ERR_ARG"):
        sp.moving_window_shift(2)
    sp.close()
