"""MI355X boosted-frame particle-in-cell step -- Python binding of ``libbfpic.so``.

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI declared in ``include/bfpic.h``.  PyTorch supplies device
memory (one workspace tensor per simulation) and the current HIP stream.

The binding refuses to run without the compiled library: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfpic.so")

FP64, FP32_SPLIT = 0, 1
BC_PERIODIC, BC_MUR = 0, 1
LOAD_RANDOM, LOAD_CENTERED = 0, 1
GATHER_MOMENTUM, GATHER_ENERGY = 0, 1
COMP = {"Ex": 0, "Ey": 1, "Ez": 2, "Bx": 3, "By": 4, "Bz": 5, "Jx": 6, "Jy": 7, "Jz": 8}
TIMER = {"gpd_tiled": 0, "gpd_global": 1, "fold_filter": 2, "yee": 3, "sort": 4,
         "inject": 5, "window": 6}
ERRORS = {-1: "ERR_ARG", -2: "ERR_CAPACITY", -3: "ERR_HIP", -4: "ERR_STATE",
          -5: "ERR_UNSUPPORTED"}


class BfpicError(RuntimeError):
    pass


class Config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nz", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("dz", C.c_double), ("dx", C.c_double), ("dy", C.c_double), ("cfl", C.c_double),
                ("shape_order", C.c_int32), ("filter_passes", C.c_int32),
                ("filter_compensate", C.c_int32), ("precision", C.c_int32),
                ("deterministic", C.c_int32), ("z_boundary", C.c_int32), ("ppc", C.c_int32),
                ("load", C.c_int32), ("sort_interval", C.c_int32), ("seed", C.c_uint64),
                ("beta_window", C.c_double), ("auto_window", C.c_int32),
                ("gather_form", C.c_int32)]


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


class Sizes(C.Structure):
    _fields_ = [("workspace_bytes", C.c_int64), ("field_bytes", C.c_int64),
                ("particle_bytes", C.c_int64), ("scratch_bytes", C.c_int64)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("window_cells", C.c_double),
                ("drift_cells", C.c_double), ("ue", C.c_double), ("ub", C.c_double),
                ("ukin", C.c_double), ("ukin_drift", C.c_double), ("wake_amp", C.c_double),
                ("gauss_res", C.c_double), ("charge", C.c_double), ("live", C.c_int64),
                ("nan_flag", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Loss(C.Structure):
    _fields_ = [("step_first", C.c_int32), ("step_last", C.c_int32), ("i0", C.c_int32),
                ("i1", C.c_int32), ("j0", C.c_int32), ("j1", C.c_int32),
                ("witness_weight", C.c_double), ("k0", C.c_int32), ("k1", C.c_int32)]


class AxisMeta(C.Structure):
    _fields_ = [("step", C.c_int64), ("t_prime", C.c_double), ("z0_prime", C.c_double),
                ("dz_prime", C.c_double), ("n", C.c_int32), ("gamma_b", C.c_double),
                ("beta_b", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

EXPORTS = ["bfpic_beta", "bfpic_drift_u", "bfpic_group_gamma", "bfpic_boosted_group_beta",
           "bfpic_boosted_dz", "bfpic_yee_dt", "bfpic_query_sizes", "bfpic_create",
           "bfpic_destroy", "bfpic_last_error", "init_boosted_plasma", "pic_step",
           "moving_window_shift", "bfpic_window_due", "diagnostics", "diagnostics_noalloc",
           "bfpic_get_field",
           "bfpic_set_field", "bfpic_num_slots", "bfpic_get_particles", "bfpic_sort",
           "bfpic_last_sort", "bfpic_sort_permutation", "bfpic_tile_shape", "bfpic_kernel_timing", "bfpic_kernel_time",
           "bfpic_adjoint_tape_bytes", "bfpic_forward_loss", "pic_step_adjoint",
           "bfpic_adjoint_per_direction", "bfpic_antenna",
           "bfpic_axis_record", "bfpic_back_transform", "bfpic_axis_spectrum",
           "bfpic_witness_bind", "bfpic_witness_lab", "bfpic_state_bytes", "pic_save",
           "pic_load"]


def lib():
    """Load the compiled library (raises if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise BfpicError(f"{LIB_PATH} is missing: run __graft_entry__.build() (no CPU fallback)")
    # torch's HIP runtime is loaded first, so that the library binds to the
    # same runtime torch allocates device memory with
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    d, i32, i64, p = C.c_double, C.c_int32, C.c_int64, C.c_void_p
    sig = {
        "bfpic_beta": (d, [d]), "bfpic_drift_u": (d, [d]), "bfpic_group_gamma": (d, [d]),
        "bfpic_boosted_group_beta": (d, [d, d]), "bfpic_boosted_dz": (d, [d, d, d]),
        "bfpic_yee_dt": (d, [i32, d, d, d, d]),
        "bfpic_query_sizes": (C.c_int, [C.POINTER(Config), i64, C.POINTER(Sizes)]),
        "bfpic_create": (C.c_int, [C.POINTER(Config), i64, p, i64, p, C.POINTER(p)]),
        "bfpic_destroy": (None, [p]), "bfpic_last_error": (C.c_char_p, [p]),
        "init_boosted_plasma": (C.c_int, [p, d, C.POINTER(Density), C.POINTER(Laser)]),
        "pic_step": (C.c_int, [p, i32]), "moving_window_shift": (C.c_int, [p, i32]),
        "bfpic_window_due": (C.c_int, [p, C.POINTER(i32)]),
        "diagnostics": (C.c_int, [p, C.c_uint32, C.POINTER(Diag), p]),
        "diagnostics_noalloc": (C.c_int, [p, C.c_uint32, C.POINTER(Diag), p]),
        "bfpic_get_field": (C.c_int, [p, i32, p]), "bfpic_set_field": (C.c_int, [p, i32, p]),
        "bfpic_num_slots": (C.c_int, [p, C.POINTER(i64)]),
        "bfpic_get_particles": (C.c_int, [p] * 9),
        "bfpic_sort": (C.c_int, [p]),
        "bfpic_last_sort": (C.c_int, [p, p, p, p, C.POINTER(i64), C.POINTER(i64),
                                      C.POINTER(i64), C.POINTER(i32)]),
        "bfpic_sort_permutation": (C.c_int, [p, p, C.POINTER(i64)]),
        "bfpic_tile_shape": (C.c_int, [p, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
        "bfpic_kernel_timing": (C.c_int, [p, i32]),
        "bfpic_kernel_time": (C.c_int, [p, i32, C.POINTER(d), C.POINTER(i64)]),
        "bfpic_adjoint_tape_bytes": (C.c_int, [p, i32, i32, C.POINTER(i64)]),
        "bfpic_forward_loss": (C.c_int, [p, i32, i32, C.POINTER(Loss), p, i64, C.POINTER(d)]),
        "pic_step_adjoint": (C.c_int, [p, C.POINTER(d), C.POINTER(d), i32]),
        "bfpic_adjoint_per_direction": (C.c_int, [p, i32]),
        "bfpic_antenna": (C.c_int, [p, C.POINTER(Laser), i32]),
        "bfpic_axis_record": (C.c_int, [p, i32, p, C.POINTER(AxisMeta)]),
        "bfpic_back_transform": (C.c_int, [p, p, p, p, i64, i32, d, d, d, d, i32, d, d, i32, d,
                                           p]),
        "bfpic_axis_spectrum": (C.c_int, [p, p, i64, i32, i32, p]),
        "bfpic_witness_bind": (C.c_int, [p, i32, p]),
        "bfpic_witness_lab": (C.c_int, [p, p]),
        "bfpic_state_bytes": (C.c_int, [p, C.POINTER(i64)]),
        "pic_save": (C.c_int, [p, p, i64]), "pic_load": (C.c_int, [p, p, i64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def beta(g): return lib().bfpic_beta(g)
def drift_u(g): return lib().bfpic_drift_u(g)
def group_gamma(n): return lib().bfpic_group_gamma(n)
def boosted_group_beta(g, n): return lib().bfpic_boosted_group_beta(g, n)
def boosted_dz(g, lam0, cells): return lib().bfpic_boosted_dz(g, lam0, cells)
def yee_dt(dim, dz, dx, dy, cfl): return lib().bfpic_yee_dt(dim, dz, dx, dy, cfl)


def make_config(**kw) -> Config:
    c = Config()
    base = dict(dim=2, nz=64, nx=32, ny=1, dz=1.0, dx=1.0, dy=1.0, cfl=0.95, shape_order=1,
                filter_passes=0, filter_compensate=0, precision=FP64, deterministic=0,
                z_boundary=BC_PERIODIC, ppc=1, load=LOAD_RANDOM, sort_interval=20, seed=0,
                beta_window=0.0, auto_window=0, gather_form=GATHER_MOMENTUM)
    base.update(kw)
    for k, v in base.items():
        setattr(c, k, v)
    return c


def make_laser(**kw) -> Laser:
    L = Laser()
    base = dict(a0=0.0, w0=0.0, L=0.0, z_center=0.0, z_focus=0.0, phase=0.0, collimated=0,
                images_z=0, images_x=0, images_y=0)
    base.update(kw)
    for k, v in base.items():
        setattr(L, k, v)
    return L


def _check(rc, h=None):
    if rc != 0:
        msg = lib().bfpic_last_error(h).decode() if h else ""
        raise BfpicError(f"{ERRORS.get(rc, rc)}: {msg}")


class Simulation:
    """A boosted-frame PIC run on the current torch device and stream."""

    def __init__(self, cfg: Config, capacity: int, device=None):
        import torch
        self.cfg = cfg
        self.capacity = int(capacity)
        sz = Sizes()
        _check(lib().bfpic_query_sizes(C.byref(cfg), self.capacity, C.byref(sz)))
        self.sizes = sz
        self.device = torch.device(device or "cuda")
        self.workspace = torch.empty(sz.workspace_bytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib().bfpic_create(C.byref(cfg), self.capacity,
                                  C.c_void_p(self.workspace.data_ptr()), sz.workspace_bytes,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        # held here so that close() still works while the interpreter shuts
        # down and module globals are already cleared
        self._destroy = lib().bfpic_destroy
        ny = cfg.ny if cfg.dim == 3 else 1
        self.field_shape = (cfg.nz + 1, cfg.nx, ny)
        self.dt = yee_dt(cfg.dim, cfg.dz, cfg.dx, cfg.dy, cfg.cfl)

    def close(self):
        h = getattr(self, "h", None)
        if h:
            self.h = None
            self._destroy(h)

    def __del__(self):
        self.close()

    # ---- the four entry points of the method ----
    def init_boosted_plasma(self, gamma_boost, n_uniform=None, knots_z=None, knots_n=None,
                            du=(0.0, 0.0, 0.0), laser: Laser | None = None, channel=None):
        dens = None
        if n_uniform is not None or knots_z is not None:
            dens = Density()
            dens.n_uniform = 0.0 if n_uniform is None else float(n_uniform)
            dens.du[:] = [float(v) for v in du]
            if channel is not None:  # (depth, radius): n (1 + depth r^2 / radius^2)
                dens.channel_depth, dens.channel_radius = (float(v) for v in channel)
            self._knots = None
            if knots_z is not None:
                kz = (C.c_double * len(knots_z))(*knots_z)
                kn = (C.c_double * len(knots_n))(*knots_n)
                self._knots = (kz, kn)
                dens.nknots = len(knots_z)
                dens.z_lab = C.cast(kz, C.POINTER(C.c_double))
                dens.n = C.cast(kn, C.POINTER(C.c_double))
        _check(lib().init_boosted_plasma(self.h, float(gamma_boost),
                                         C.byref(dens) if dens is not None else None,
                                         C.byref(laser) if laser is not None else None), self.h)
        self._wit = None  # init unbinds the witnesses

    def antenna(self, laser: Laser | None = None, row=0):
        """Laser antenna on grid row `row` emitting `laser` (None removes it)."""
        self._antenna = laser
        _check(lib().bfpic_antenna(self.h, C.byref(laser) if laser is not None else None,
                                   int(row)), self.h)

    def pic_step(self, nsteps=1):
        _check(lib().pic_step(self.h, int(nsteps)), self.h)

    def moving_window_shift(self, ncells):
        _check(lib().moving_window_shift(self.h, int(ncells)), self.h)

    def window_due(self) -> int:
        n = C.c_int32()
        _check(lib().bfpic_window_due(self.h, C.byref(n)), self.h)
        return n.value

    def diagnostics(self, lineout=False, noalloc=False) -> dict:
        """FP64 diagnostics; noalloc=True calls diagnostics_noalloc (static
        device scratch) instead of diagnostics."""
        import torch
        d = Diag()
        lo = torch.zeros(self.cfg.nz, dtype=torch.float64, device=self.device) if lineout else None
        fn = lib().diagnostics_noalloc if noalloc else lib().diagnostics
        _check(fn(self.h, 0xFFFFFFFF, C.byref(d),
                  C.c_void_p(lo.data_ptr()) if lo is not None else None), self.h)
        out = d.as_dict()
        if lineout:
            out["lineout"] = lo.cpu().numpy()
        return out

    # ---- state access ----
    def axis_record(self, frame=1):
        """On-axis transverse laser field (rows 0..nz): frame 0 boosted E'_y,
        frame 1 the lab field gamma_b (E'_y - beta_b B'_x).  Returns (device
        tensor, meta dict)."""
        import torch
        m = AxisMeta()
        out = torch.empty(self.cfg.nz + 1, dtype=torch.float64, device=self.device)
        _check(lib().bfpic_axis_record(self.h, int(frame), C.c_void_p(out.data_ptr()),
                                       C.byref(m)), self.h)
        return out, m.as_dict()

    def back_transform(self, rec, t_prime, z0_prime, dz_prime, gamma_b, t0, dt, nt, zeta0,
                       dzeta, nzeta, v_window):
        """Lab-frame values (nt x nzeta) of a record history, see
        bfpic_back_transform.  rec: (nrec, n) device tensor (FP64)."""
        import torch
        rec = torch.as_tensor(rec, dtype=torch.float64, device=self.device).contiguous()
        tp = torch.as_tensor(t_prime, dtype=torch.float64, device=self.device).contiguous()
        z0 = torch.as_tensor(z0_prime, dtype=torch.float64, device=self.device).contiguous()
        out = torch.empty((int(nt), int(nzeta)), dtype=torch.float64, device=self.device)
        _check(lib().bfpic_back_transform(
            self.h, C.c_void_p(rec.data_ptr()), C.c_void_p(tp.data_ptr()),
            C.c_void_p(z0.data_ptr()), rec.shape[0], rec.shape[1], float(dz_prime),
            float(gamma_b), float(t0), float(dt), int(nt), float(zeta0), float(dzeta),
            int(nzeta), float(v_window), C.c_void_p(out.data_ptr())), self.h)
        return out

    def axis_spectrum(self, rec, m):
        """|DFT|^2 (q = 0..m/2) of each record zero-padded to m points."""
        import torch
        rec = torch.as_tensor(rec, dtype=torch.float64, device=self.device).contiguous()
        out = torch.empty((rec.shape[0], int(m) // 2 + 1), dtype=torch.float64, device=self.device)
        _check(lib().bfpic_axis_spectrum(self.h, C.c_void_p(rec.data_ptr()), rec.shape[0],
                                         rec.shape[1], int(m), C.c_void_p(out.data_ptr())), self.h)
        return out

    def witness_bind(self, state):
        """Binds a (n, 6) FP64 device tensor of witness electrons (z, x, y,
        u_z, u_x, u_y), advanced in place by every pic_step; None unbinds."""
        if state is None:
            _check(lib().bfpic_witness_bind(self.h, 0, None), self.h)
            self._wit = None
            return
        import torch
        if (state.dtype != torch.float64 or state.device.type != "cuda" or state.dim() != 2
                or state.shape[1] != 6 or not state.is_contiguous()):
            raise BfpicError("witness state: contiguous (n, 6) float64 device tensor")
        _check(lib().bfpic_witness_bind(self.h, state.shape[0], C.c_void_p(state.data_ptr())),
               self.h)
        self._wit = state

    def witness_lab(self):
        """(n, 4) device tensor: lab t, z, gamma, u_z of the bound witnesses."""
        import torch
        n = 0 if getattr(self, "_wit", None) is None else self._wit.shape[0]
        out = torch.empty((max(n, 1), 4), dtype=torch.float64, device=self.device)
        _check(lib().bfpic_witness_lab(self.h, C.c_void_p(out.data_ptr())), self.h)
        return out[:n]

    def save(self):
        """The simulation state as a uint8 device tensor (see pic_save)."""
        import torch
        nb = C.c_int64()
        _check(lib().bfpic_state_bytes(self.h, C.byref(nb)), self.h)
        blob = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        _check(lib().pic_save(self.h, C.c_void_p(blob.data_ptr()), nb.value), self.h)
        return blob

    def load(self, blob):
        """Resumes from a state saved by `save` (same configuration)."""
        import torch
        if not isinstance(blob, torch.Tensor) or blob.dtype != torch.uint8 or blob.dim() != 1:
            raise BfpicError("state blob: a 1-D uint8 tensor written by save()")
        blob = blob.to(self.device).contiguous()
        _check(lib().pic_load(self.h, C.c_void_p(blob.data_ptr()), blob.numel()), self.h)

    def get_field(self, comp):
        import torch
        comp = COMP.get(comp, comp)
        out = torch.empty(self.field_shape, dtype=torch.float64, device=self.device)
        _check(lib().bfpic_get_field(self.h, comp, C.c_void_p(out.data_ptr())), self.h)
        return out

    def set_field(self, comp, arr):
        import torch
        comp = COMP.get(comp, comp)
        t = torch.as_tensor(arr, dtype=torch.float64).to(self.device).expand(self.field_shape)
        t = t.contiguous()
        _check(lib().bfpic_set_field(self.h, comp, C.c_void_p(t.data_ptr())), self.h)
        self.stream.synchronize()

    def num_slots(self) -> int:
        n = C.c_int64()
        _check(lib().bfpic_num_slots(self.h, C.byref(n)), self.h)
        return n.value

    def particles(self) -> dict:
        import torch
        n = self.num_slots()
        names = ["z", "x", "y", "ux", "uy", "uz", "w"]
        out = {k: torch.zeros(max(n, 1), dtype=torch.float64, device=self.device) for k in names}
        out["id"] = torch.zeros(max(n, 1), dtype=torch.int32, device=self.device)
        _check(lib().bfpic_get_particles(self.h, *[C.c_void_p(out[k].data_ptr()) for k in names],
                                         C.c_void_p(out["id"].data_ptr())), self.h)
        return {k: v[:n].cpu().numpy() for k, v in out.items()}

    def sort(self):
        _check(lib().bfpic_sort(self.h), self.h)

    def last_sort(self) -> dict:
        import torch
        n_cap = max(self.capacity, 1)
        key = torch.empty(n_cap, dtype=torch.int32, device=self.device)
        pid = torch.empty(n_cap, dtype=torch.int32, device=self.device)
        perm = torch.empty(n_cap, dtype=torch.int32, device=self.device)
        n, nl, tzmin, ntz = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().bfpic_last_sort(self.h, C.c_void_p(key.data_ptr()), C.c_void_p(pid.data_ptr()),
                                     C.c_void_p(perm.data_ptr()), C.byref(n), C.byref(nl),
                                     C.byref(tzmin), C.byref(ntz)), self.h)
        return {"key": key[: n.value].cpu().numpy(), "id": pid[: n.value].cpu().numpy(),
                "perm": perm[: nl.value].cpu().numpy(), "tz_min": tzmin.value, "ntz": ntz.value}

    def sort_permutation(self):
        """perm[d] = source slot of destination d of the last sort (live only)."""
        import torch
        perm = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=self.device)
        nl = C.c_int64()
        _check(lib().bfpic_sort_permutation(self.h, C.c_void_p(perm.data_ptr()), C.byref(nl)),
               self.h)
        return perm[: nl.value].cpu().numpy()

    def tile_shape(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().bfpic_tile_shape(self.h, C.byref(a), C.byref(b), C.byref(c)), self.h)
        return a.value, b.value, c.value

    def kernel_timing(self, enable=True):
        _check(lib().bfpic_kernel_timing(self.h, 1 if enable else 0), self.h)

    def kernel_time(self, cls) -> tuple:
        cls = TIMER.get(cls, cls)
        ms, n = C.c_double(), C.c_int64()
        _check(lib().bfpic_kernel_time(self.h, cls, C.byref(ms), C.byref(n)), self.h)
        return ms.value, n.value

    # ---- adjoint ----
    def forward_loss(self, nsteps, interval, step_first, step_last, box,
                     witness_weight=0.0) -> float:
        """Taped run of `nsteps` steps from the state right after init, with a
        checkpoint every `interval` steps; returns the loss: the mean of Ez over
        the node box (i0, i1, j0, j1), in 3D (i0, i1, j0, j1, k0, k1), averaged
        over steps step_first..step_last,
        plus witness_weight times the mean lab energy of the bound witnesses
        after the last step."""
        import torch
        nb = C.c_int64()
        _check(lib().bfpic_adjoint_tape_bytes(self.h, nsteps, interval, C.byref(nb)), self.h)
        self.tape = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        i0, i1, j0, j1, k0, k1 = tuple(box) + (0, 0) if len(box) == 4 else tuple(box)
        loss = Loss(step_first, step_last, i0, i1, j0, j1, float(witness_weight), k0, k1)
        out = C.c_double()
        _check(lib().bfpic_forward_loss(self.h, nsteps, interval, C.byref(loss),
                                        C.c_void_p(self.tape.data_ptr()), nb.value,
                                        C.byref(out)), self.h)
        return out.value

    def adjoint_per_direction(self, enable=True):
        """Selects the per-direction reverse particle step (the reference)."""
        _check(lib().bfpic_adjoint_per_direction(self.h, int(bool(enable))), self.h)

    def adjoint(self, nknots=1):
        """Reverse sweep of the last taped run: (dL/da0, dL/dn) with dL/dn per
        density knot (one value for a uniform density)."""
        da0 = C.c_double()
        dn = (C.c_double * max(nknots, 1))()
        _check(lib().pic_step_adjoint(self.h, C.byref(da0), dn, max(nknots, 1)), self.h)
        return da0.value, [dn[m] for m in range(max(nknots, 1))]
