"""Oracle of witness electrons: test particles pushed by the fields of a run.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/`` may import
it.  Plain FP64 numpy, written from the definitions:

* gather: each field component from its own staggered nodes, weighted by the
  deposit's shape (S of order 1 or 2) of the distance to each node;
* push: the relativistic Boris step of the oracle (``orc_boris``), q = -1;
* move: position += v dt / d per axis (grid cells), x (and y) periodic, z
  periodic in a periodic box;
* lab view (section "Modeling of up to 1 TeV stages": energy gain of the
  accelerated beam against lab position): the witness's event
  (t', z' = (z + window) dz') and momentum boosted back to the lab frame,
  t = g (t' + b z'), z = g (z' + b t'), gamma = g (gamma' + b u'_z),
  u_z = g (u'_z + b gamma').

A witness row is (z, x, y, u_z, u_x, u_y): position in grid cells relative to
the window, momentum in the calculation frame.
"""
from __future__ import annotations

import math

import numpy as np

from . import Sim, beta_of_gamma, boris, shape

# node offsets (z, x, y) of each component in cells
STAGGER = {"Ex": (0.0, 0.5, 0.0), "Ey": (0.0, 0.0, 0.5), "Ez": (0.5, 0.0, 0.0),
           "Bx": (0.5, 0.0, 0.5), "By": (0.5, 0.5, 0.0), "Bz": (0.0, 0.5, 0.5)}


def fields(sim: Sim) -> dict:
    return {c: sim.get_field(c) for c in STAGGER}


def gather(F: dict, sim: Sim, z: float, x: float, y: float = 0.0):
    """E, B (x, y, z order) at the position, from component arrays of rows
    0..nz (rows beyond them hold zero fields; periodic z wraps)."""
    c = sim.cfg
    dim = c.dim
    periodic = c.zbc == 0
    out = {}
    for name, (sz, sx, sy) in STAGGER.items():
        # energy-conserving (Galerkin) form: one order lower along each axis
        # on which the component sits at half-integer nodes
        oz, ox, oy = (c.order - 1 if (c.gather == 1 and s == 0.5) else c.order
                      for s in (sz, sx, sy))
        A = F[name]
        acc = 0.0
        for i in range(math.floor(z - sz) - 2, math.floor(z - sz) + 3):
            wz = shape(oz, z - (i + sz))
            if wz == 0.0:
                continue
            if periodic:
                ii = i % c.nz
            elif 0 <= i <= c.nz:
                ii = i
            else:
                continue
            for j in range(math.floor(x - sx) - 2, math.floor(x - sx) + 3):
                wx = shape(ox, x - (j + sx))
                if wx == 0.0:
                    continue
                jj = j % c.nx
                if dim == 3:
                    for k in range(math.floor(y - sy) - 2, math.floor(y - sy) + 3):
                        wy = shape(oy, y - (k + sy))
                        if wy != 0.0:
                            acc += wz * wx * wy * A[ii, jj, k % c.ny]
                else:
                    acc += wz * wx * A[ii, jj, 0]
        out[name] = acc
    return [out["Ex"], out["Ey"], out["Ez"]], [out["Bx"], out["By"], out["Bz"]]


def push(sim: Sim, W: np.ndarray, F: dict | None = None) -> None:
    """One step of every witness in W (n x 6, updated in place) through the
    fields F (default: the present fields of sim)."""
    c = sim.cfg
    F = fields(sim) if F is None else F
    for r in range(len(W)):
        z, x, y, uz, ux, uy = W[r]
        E, B = gather(F, sim, z, x, y)
        u = boris(-1.0, c.dt, E, B, [ux, uy, uz])
        g = math.sqrt(1.0 + u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
        z += u[2] / g * c.dt / c.dz
        if c.zbc == 0:
            z %= c.nz
        x = (x + u[0] / g * c.dt / c.dx) % c.nx
        if c.dim == 3:
            y = (y + u[1] / g * c.dt / c.dy) % c.ny
        W[r] = (z, x, y, u[2], u[0], u[1])


def lab(W: np.ndarray, t_prime: float, window_cells: float, dz: float, gamma_b: float):
    """Rows (t, z, gamma, u_z) in the lab frame."""
    b = beta_of_gamma(gamma_b)
    out = np.zeros((len(W), 4))
    for r, (z, x, y, uz, ux, uy) in enumerate(W):
        zp = (z + window_cells) * dz
        gp = math.sqrt(1.0 + uz * uz + ux * ux + uy * uy)
        out[r] = (gamma_b * (t_prime + b * zp), gamma_b * (zp + b * t_prime),
                  gamma_b * (gp + b * uz), gamma_b * (uz + b * gp))
    return out
