"""The C-ABI library, checked without a GPU: it loads, exports every symbol the
header declares, sizes its workspace on the host, rejects bad configurations,
and its boost helper agrees with the oracle's independent copy."""
import ctypes
import math
import os
import re

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfpic.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", src)
    return sorted({n for n in names if n not in ("if", "sizeof")})


@pytest.fixture(scope="module")
def P():
    import paper_1011_0917_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1011_0917_amd import build
        build.build()
    P.lib()
    return P


def test_exports_every_declared_symbol(P):
    L = ctypes.CDLL(P.LIB_PATH)
    names = _declared()
    assert "init_boosted_plasma" in names and "pic_step" in names
    assert "moving_window_shift" in names and "diagnostics" in names
    for n in names:
        assert hasattr(L, n), n


def test_binding_wraps_every_export(P):
    assert set(_declared()) <= set(P.EXPORTS)


def test_boost_helper_agrees_with_oracle(P):
    for g in (1.0, 13.0, 130.0, 1300.0):
        assert P.beta(g) == pytest.approx(O.beta_of_gamma(g), rel=1e-15, abs=0)
        assert P.drift_u(g) == pytest.approx(O.drift_u(g), rel=1e-15, abs=0)
        assert P.boosted_dz(g, 2 * math.pi, 16) == pytest.approx(O.boosted_dz(g, 2 * math.pi, 16),
                                                                 rel=1e-15)
    for g, n in ((13.0, 1e-3), (130.0, 1e-4), (100.0, 3e-4)):
        assert P.boosted_group_beta(g, n) == pytest.approx(O.boosted_group_beta(g, n), rel=1e-13)
    assert P.yee_dt(3, 1.0, 0.5, 0.4, 0.95) == pytest.approx(O.yee_dt(3, 1.0, 0.5, 0.4, 0.95))


def test_query_sizes_and_bad_configs(P):
    c = P.make_config(dim=2, nz=8192, nx=512, precision=P.FP32_SPLIT, ppc=8,
                      z_boundary=P.BC_MUR, filter_passes=4, filter_compensate=1)
    s = P.Sizes()
    assert P.lib().bfpic_query_sizes(ctypes.byref(c), 34_000_000, ctypes.byref(s)) == 0
    # particles: two sort buffers of id + 2 xi + 3 du + w (4 bytes each)
    assert s.particle_bytes >= 2 * 34_000_000 * 28
    assert s.workspace_bytes == s.field_bytes + s.particle_bytes + s.scratch_bytes
    for bad in (dict(dim=4), dict(cfl=1.2), dict(shape_order=3), dict(ppc=0), dict(nz=2)):
        cb = P.make_config(**bad)
        assert P.lib().bfpic_query_sizes(ctypes.byref(cb), 10, ctypes.byref(s)) == -1
    # deterministic mode: accepted; the overflow grid and tile current scratch
    # hold int64 sums, so an FP32 run needs more workspace
    cd = P.make_config(dim=2, nz=8192, nx=512, precision=P.FP32_SPLIT, ppc=8,
                       z_boundary=P.BC_MUR, filter_passes=4, filter_compensate=1,
                       deterministic=1)
    sd = P.Sizes()
    assert P.lib().bfpic_query_sizes(ctypes.byref(cd), 34_000_000, ctypes.byref(sd)) == 0
    assert sd.field_bytes > s.field_bytes and sd.scratch_bytes > s.scratch_bytes
    assert sd.particle_bytes == s.particle_bytes


def test_create_rejects_small_workspace(P):
    c = P.make_config()
    h = ctypes.c_void_p()
    rc = P.lib().bfpic_create(ctypes.byref(c), 100, ctypes.c_void_p(256), 16, None, ctypes.byref(h))
    assert rc == -1 and not h.value


def test_workloads_resolve_identically_on_both_sides(P):
    from workloads import WORKLOADS, resolve_gpu, resolve_oracle
    for name, W in WORKLOADS.items():
        cfg, init, _ = resolve_gpu(W)
        kw, oinit = resolve_oracle(W)
        assert cfg.dz == pytest.approx(kw["dz"], rel=1e-15)
        assert cfg.beta_window == pytest.approx(kw["beta_window"], rel=1e-13, abs=1e-16)
        assert P.yee_dt(cfg.dim, cfg.dz, cfg.dx, cfg.dy, cfg.cfl) == pytest.approx(kw["dt"], rel=1e-15)
        assert init["laser"].z_center == pytest.approx(oinit["laser"].z_center, rel=1e-14)


STRUCTS = {"Config": "bfpic_config", "Density": "bfpic_density", "Laser": "bfpic_laser",
           "Loss": "bfpic_loss", "Sizes": "bfpic_sizes", "Diag": "bfpic_diag",
           "AxisMeta": "bfpic_axis_meta"}


def _check_layouts(mod, structs, header_dir, header, tmp_path):
    """Size and field offsets of each ctypes structure of `mod` against its C
    struct, read from a program that gcc compiles against the header."""
    import subprocess
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{header}"',
             "int main(void) {"]
    for py, c in structs.items():
        lines.append(f'  printf("{py} size %zu\\n", sizeof({c}));')
        for f, _ in getattr(mod, py)._fields_:
            lines.append(f'  printf("{py} {f} %zu\\n", offsetof({c}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", header_dir, "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    assert out
    for line in out.splitlines():
        py, field, value = line.split()
        cls = getattr(mod, py)
        want = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert int(value) == want, (py, field, value, want)


def test_binding_structs_match_the_header(P, tmp_path):
    _check_layouts(P, STRUCTS, os.path.join(ROOT, "include"), "bfpic.h", tmp_path)


def test_oracle_structs_match_its_header(tmp_path):
    structs = {"Config": "orc_config", "Density": "orc_density", "Laser": "orc_laser",
               "Diag": "orc_diag"}
    _check_layouts(O, structs, os.path.join(ROOT, "oracle"), "pic_oracle.h", tmp_path)


def test_query_and_create_share_the_capacity_bound(P):
    c = P.make_config()
    s = P.Sizes()
    assert P.lib().bfpic_query_sizes(ctypes.byref(c), 2 ** 31 - 1, ctypes.byref(s)) == 0
    assert P.lib().bfpic_query_sizes(ctypes.byref(c), 2 ** 31, ctypes.byref(s)) == -1
    h = ctypes.c_void_p()
    rc = P.lib().bfpic_create(ctypes.byref(c), 2 ** 31, ctypes.c_void_p(256), 1 << 40, None,
                              ctypes.byref(h))
    assert rc == -1 and not h.value


def _host_ctx(P, buf_keep, **kw):
    """A context over a host buffer standing in for the workspace.  Only calls
    that fail their argument checks, which run before any device work, may be
    made on it."""
    c = P.make_config(**kw)
    s = P.Sizes()
    cap = kw.get("nz", 64) * kw.get("nx", 32) * kw.get("ppc", 1)
    assert P.lib().bfpic_query_sizes(ctypes.byref(c), cap, ctypes.byref(s)) == 0
    buf = ctypes.create_string_buffer(s.workspace_bytes + 256)
    buf_keep.append(buf)
    base = (ctypes.addressof(buf) + 255) & ~255
    h = ctypes.c_void_p()
    rc = P.lib().bfpic_create(ctypes.byref(c), cap, ctypes.c_void_p(base), s.workspace_bytes,
                              None, ctypes.byref(h))
    if rc != 0:
        pytest.skip("context creation needs the HIP runtime here")
    return h, cap


def test_init_rejects_bad_density_before_any_device_work(P):
    keep = []
    h, cap = _host_ctx(P, keep, nz=16, nx=8, ppc=2, z_boundary=P.BC_MUR)
    L = P.lib()
    try:
        d = P.Density()
        kz = (ctypes.c_double * 33)(*[float(i) for i in range(33)])
        kn = (ctypes.c_double * 33)(*([1e-3] * 33))
        d.nknots, d.z_lab, d.n = 33, ctypes.cast(kz, ctypes.POINTER(ctypes.c_double)), \
            ctypes.cast(kn, ctypes.POINTER(ctypes.c_double))
        assert L.init_boosted_plasma(h, 13.0, ctypes.byref(d), None) == -1
        d.nknots = 3
        kz[1] = kz[0]  # not increasing
        assert L.init_boosted_plasma(h, 13.0, ctypes.byref(d), None) == -1
        kz[1] = 1.0
        d.channel_depth, d.channel_radius = 0.5, 0.0
        assert L.init_boosted_plasma(h, 13.0, ctypes.byref(d), None) == -1
        # nothing was initialised: stepping is still out of order
        assert L.pic_step(h, 1) == -4
    finally:
        L.bfpic_destroy(h)


def test_init_rejects_capacity_before_any_device_work(P):
    L = P.lib()
    # a capacity below the box's particles
    c = P.make_config(nz=16, nx=8, ppc=2, z_boundary=P.BC_MUR)
    s = P.Sizes()
    assert L.bfpic_query_sizes(ctypes.byref(c), 100, ctypes.byref(s)) == 0
    buf = ctypes.create_string_buffer(s.workspace_bytes + 256)
    base = (ctypes.addressof(buf) + 255) & ~255
    h = ctypes.c_void_p()
    if L.bfpic_create(ctypes.byref(c), 100, ctypes.c_void_p(base), s.workspace_bytes, None,
                      ctypes.byref(h)) != 0:
        pytest.skip("context creation needs the HIP runtime here")
    try:
        d = P.Density()
        d.n_uniform = 1e-3
        assert L.init_boosted_plasma(h, 13.0, ctypes.byref(d), None) == -2
        assert b"capacity" in L.bfpic_last_error(h)
    finally:
        L.bfpic_destroy(h)
