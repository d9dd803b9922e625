"""Plain FP64 CPU particle-in-cell oracle (ctypes binding).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_1011_0917_amd``) never imports it, and the two share no code.

The C source ``pic_oracle.c`` holds the arithmetic; this module only builds it
and marshals arguments.  See the header comment of ``pic_oracle.h`` for what
the oracle computes and which method each step follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EX, EY, EZ, BX, BY, BZ, JX, JY, JZ = range(9)
COMP = {"Ex": EX, "Ey": EY, "Ez": EZ, "Bx": BX, "By": BY, "Bz": BZ,
        "Jx": JX, "Jy": JY, "Jz": JZ}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-std=c99", "-D_DEFAULT_SOURCE", "-O2", "-fPIC", "-shared",
               "-ffp-contract=off", "-fopenmp", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nz", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("dz", C.c_double), ("dx", C.c_double), ("dy", C.c_double), ("dt", C.c_double),
                ("order", C.c_int32), ("filter_passes", C.c_int32),
                ("filter_compensate", C.c_int32), ("zbc", C.c_int32), ("ppc", C.c_int32),
                ("seed", C.c_uint64), ("gamma_b", C.c_double), ("beta_window", C.c_double),
                ("auto_window", C.c_int32), ("ions", C.c_int32), ("load", C.c_int32),
                ("gather", C.c_int32)]


class Density(C.Structure):
    _fields_ = [("n_uniform", C.c_double), ("nknots", C.c_int32),
                ("z_lab", C.POINTER(C.c_double)), ("n", C.POINTER(C.c_double)),
                ("du", C.c_double * 3), ("channel_depth", C.c_double),
                ("channel_radius", C.c_double)]


class Laser(C.Structure):
    _fields_ = [("a0", C.c_double), ("w0", C.c_double), ("L", C.c_double),
                ("z_center", C.c_double), ("z_focus", C.c_double), ("phase", C.c_double),
                ("collimated", C.c_int32), ("images_z", C.c_int32), ("images_x", C.c_int32),
                ("images_y", C.c_int32)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("window_cells", C.c_double),
                ("drift_cells", C.c_double), ("ue", C.c_double), ("ub", C.c_double),
                ("ukin", C.c_double), ("ukin_drift", C.c_double), ("wake_amp", C.c_double),
                ("gauss_res", C.c_double), ("charge", C.c_double), ("live", C.c_int64),
                ("nan_flag", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        d, i32, i64, u64, p = C.c_double, C.c_int32, C.c_int64, C.c_uint64, C.c_void_p
        dp = C.POINTER(C.c_double)
        sig = {
            "orc_beta_of_gamma": (d, [d]), "orc_one_minus_beta": (d, [d]),
            "orc_drift_u": (d, [d]), "orc_group_gamma": (d, [d]),
            "orc_boosted_group_beta": (d, [d, d]), "orc_boosted_dz": (d, [d, d, d]),
            "orc_yee_dt": (d, [i32, d, d, d, d]), "orc_depletion_length": (d, [d]),
            "orc_splitmix64": (u64, [u64, u64]),
            "orc_cell_offset": (d, [u64, i64, i64, i64, i32, i32, i32, i32, i32]),
            "orc_shape": (d, [i32, d]),
            "orc_boris": (None, [d, d, dp, dp, dp]),
            "orc_sort_perm": (None, [i64, p, p, p]),
            "orc_create": (p, [C.POINTER(Config)]), "orc_destroy": (None, [p]),
            "orc_init": (C.c_int, [p, C.POINTER(Density), C.POINTER(Laser), i32]),
            "orc_step": (C.c_int, [p, i32]), "orc_window_shift": (C.c_int, [p, i32]),
            "orc_set_antenna": (C.c_int, [p, C.POINTER(Laser), i32]),
            "orc_diagnostics": (C.c_int, [p, C.POINTER(Diag), p]),
            "orc_field_size": (i64, [p]), "orc_get_field": (C.c_int, [p, i32, p]),
            "orc_set_field": (C.c_int, [p, i32, p]), "orc_num_pairs": (i64, [p]),
            "orc_get_particles": (C.c_int, [p] * 10),
            "orc_add_pair": (C.c_int, [p, d, d, d, d, d, d, d, d, d, d, i64]),
            "orc_clear_particles": (None, [p]),
            "orc_sort_keys": (C.c_int, [p, i32, i32, i32, i64, i32, p, p]),
            "orc_laser_eval": (None, [C.POINTER(Laser), i32, d, d, d, d, d, dp, dp]),
            "orc_filter_field": (C.c_int, [p, i32]),
            "orc_lab_density": (d, [p, d]), "orc_channel_factor": (d, [p, d, d]),
            "orc_set_threads": (C.c_int, [p, i32]), "orc_max_threads": (i32, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---- thin function wrappers -------------------------------------------------

def beta_of_gamma(g): return lib().orc_beta_of_gamma(g)
def one_minus_beta(g): return lib().orc_one_minus_beta(g)
def drift_u(g): return lib().orc_drift_u(g)
def group_gamma(n): return lib().orc_group_gamma(n)
def boosted_group_beta(g, n): return lib().orc_boosted_group_beta(g, n)
def boosted_dz(g, lam0, cpw): return lib().orc_boosted_dz(g, lam0, cpw)
def yee_dt(dim, dz, dx, dy, cfl): return lib().orc_yee_dt(dim, dz, dx, dy, cfl)
def depletion_length(n): return lib().orc_depletion_length(n)
def splitmix64(seed, n): return lib().orc_splitmix64(seed, n)
def shape(order, d): return lib().orc_shape(order, d)
def max_threads(): return lib().orc_max_threads()


def cell_offset(seed, k, l, j, s, axis, nx, nyy, ppc):
    return lib().orc_cell_offset(seed, k, l, j, s, axis, nx, nyy, ppc)


def boris(q, dt, E, B, u):
    E = (C.c_double * 3)(*E)
    B = (C.c_double * 3)(*B)
    uu = (C.c_double * 3)(*u)
    lib().orc_boris(q, dt, E, B, uu)
    return [uu[0], uu[1], uu[2]]


def sort_perm(keys: np.ndarray, ids: np.ndarray) -> np.ndarray:
    k = np.ascontiguousarray(keys, dtype=np.int32)
    i = np.ascontiguousarray(ids, dtype=np.int32)
    perm = np.empty(len(k), dtype=np.int32)
    lib().orc_sort_perm(len(k), _ptr(k), _ptr(i), _ptr(perm))
    return perm


def make_laser(**kw) -> Laser:
    L = Laser()
    defaults = dict(a0=0.0, w0=0.0, L=0.0, z_center=0.0, z_focus=0.0, phase=0.0,
                    collimated=0, images_z=0, images_x=0, images_y=0)
    defaults.update(kw)
    for k, v in defaults.items():
        setattr(L, k, v)
    return L


def laser_eval(laser: Laser, dim, gamma_b, zp, x, y=0.0, tp=0.0):
    A = C.c_double()
    E = C.c_double()
    lib().orc_laser_eval(C.byref(laser), dim, gamma_b, tp, zp, x, y, C.byref(A), C.byref(E))
    return A.value, E.value


class Sim:
    """One oracle simulation.  Arguments mirror ``orc_config``."""

    def __init__(self, dim=2, nz=16, nx=16, ny=1, dz=1.0, dx=1.0, dy=1.0, dt=0.5, order=1,
                 filter_passes=0, filter_compensate=0, zbc=0, ppc=1, seed=0, gamma_b=1.0,
                 beta_window=0.0, auto_window=0, ions=1, load=0, gather=0):
        c = Config(dim=dim, nz=nz, nx=nx, ny=ny if dim == 3 else 1, dz=dz, dx=dx, dy=dy, dt=dt,
                   order=order, filter_passes=filter_passes,
                   filter_compensate=filter_compensate, zbc=zbc, ppc=ppc, seed=seed,
                   gamma_b=gamma_b, beta_window=beta_window, auto_window=auto_window, ions=ions,
                   load=load, gather=gather)
        self.cfg = c
        self.h = lib().orc_create(C.byref(c))
        self.shape = (nz + 1, nx, (ny if dim == 3 else 1))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def init(self, n_uniform=None, knots_z=None, knots_n=None, laser: Laser | None = None,
             fill=True, du=(0.0, 0.0, 0.0), channel=None):
        dens = None
        self._keep = []
        if n_uniform is not None or knots_z is not None:
            dens = Density()
            dens.n_uniform = 0.0 if n_uniform is None else float(n_uniform)
            dens.du[:] = [float(v) for v in du]
            if channel is not None:
                dens.channel_depth, dens.channel_radius = (float(v) for v in channel)
            if knots_z is not None:
                kz = np.ascontiguousarray(knots_z, dtype=np.float64)
                kn = np.ascontiguousarray(knots_n, dtype=np.float64)
                self._keep += [kz, kn]
                dens.nknots = len(kz)
                dens.z_lab = kz.ctypes.data_as(C.POINTER(C.c_double))
                dens.n = kn.ctypes.data_as(C.POINTER(C.c_double))
            else:
                dens.nknots = 0
        rc = lib().orc_init(self.h, C.byref(dens) if dens is not None else None,
                            C.byref(laser) if laser is not None else None, 1 if fill else 0)
        assert rc == 0

    def step(self, n=1):
        assert lib().orc_step(self.h, n) == 0

    def set_antenna(self, laser: Laser | None, row=-1):
        """Laser antenna on grid row `row` (None removes it): each later step
        adds the current sheet that emits the laser's boosted E_y there."""
        self._antenna = laser
        rc = lib().orc_set_antenna(self.h, C.byref(laser) if laser is not None else None,
                                   int(row) if laser is not None else -1)
        assert rc == 0, "antenna row out of range"

    def window_shift(self, n):
        assert lib().orc_window_shift(self.h, n) == 0

    def diagnostics(self, lineout=False):
        d = Diag()
        lo = np.zeros(self.cfg.nz + 1, dtype=np.float64) if lineout else None
        lib().orc_diagnostics(self.h, C.byref(d), _ptr(lo) if lo is not None else None)
        out = d.as_dict()
        if lineout:
            out["lineout"] = lo[: self.cfg.nz].copy()
        return out

    def get_field(self, comp) -> np.ndarray:
        comp = COMP.get(comp, comp)
        a = np.empty(self.shape, dtype=np.float64)
        assert lib().orc_get_field(self.h, comp, _ptr(a)) == 0
        return a

    def set_field(self, comp, arr):
        comp = COMP.get(comp, comp)
        a = np.ascontiguousarray(np.broadcast_to(arr, self.shape), dtype=np.float64)
        assert lib().orc_set_field(self.h, comp, _ptr(a)) == 0

    def filter_field(self, comp):
        comp = COMP.get(comp, comp)
        assert lib().orc_filter_field(self.h, comp) == 0

    def num_pairs(self) -> int:
        return lib().orc_num_pairs(self.h)

    def particles(self) -> dict:
        n = self.num_pairs()
        names = ["ze", "xe", "ye", "uz", "ux", "uy", "zi", "w"]
        out = {k: np.empty(n, dtype=np.float64) for k in names}
        out["id"] = np.empty(n, dtype=np.int64)
        lib().orc_get_particles(self.h, *[_ptr(out[k]) for k in names], _ptr(out["id"]))
        return out

    def add_pair(self, ze, xe, ye, uz, ux, uy, zi, xi, yi, w, pid):
        lib().orc_add_pair(self.h, ze, xe, ye, uz, ux, uy, zi, xi, yi, w, pid)

    def clear_particles(self):
        lib().orc_clear_particles(self.h)

    def set_threads(self, n: int):
        """Threads of the particle loop (per-thread current buffers)."""
        assert lib().orc_set_threads(self.h, int(n)) == 0

    def lab_density(self, z_lab: float) -> float:
        return lib().orc_lab_density(self.h, float(z_lab))

    def channel_factor(self, x: float, y: float = 0.0) -> float:
        return lib().orc_channel_factor(self.h, float(x), float(y))

    def sort_keys(self, tz, tx, ty, tz_min, ntz):
        n = self.num_pairs()
        key = np.empty(n, dtype=np.int32)
        pid = np.empty(n, dtype=np.int32)
        lib().orc_sort_keys(self.h, tz, tx, ty, tz_min, ntz, _ptr(key), _ptr(pid))
        return key, pid
