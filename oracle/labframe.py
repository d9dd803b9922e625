"""Oracle of the lab-frame and spectral diagnostics of the on-axis laser field.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/`` may import
it.  Plain, slow FP64 numpy written from the definitions:

* record (section "Effect of the hyperbolic rotation in Minkowski space",
  Fig. 2: histories of the transverse laser field on axis): the boosted E'_y on
  the axis row, or the lab-frame field at the same event.  The transverse
  fields transform as E_y = gamma (E'_y - beta B'_x) from a frame moving at
  +beta along z (c = 1);
* back_transform (same section: boosted data shown in the laboratory-frame
  moving window): each lab event (t, z = zeta + v_w t) is mapped to the boosted
  event t' = gamma (t - beta z), z' = gamma (z - beta t) and read from the
  record history by linear interpolation in z' and then in t';
* spectrum (section "Mitigation of a numerical instability", Fig. 3: spectral
  content history of the on-axis laser field): |DFT|^2 of each record along z.
"""
from __future__ import annotations

import math

import numpy as np

from . import Sim, beta_of_gamma


def record(sim: Sim, frame: int, gamma_b: float) -> np.ndarray:
    """Axis row (j = nx/2, k = ny/2), rows 0..nz.  frame 0: E'_y; frame 1:
    gamma_b (E'_y - beta_b B'_x), B'_x (held at half rows i + 1/2) averaged
    onto row i.  Rows outside the B_x domain count as zero (open z) or wrap
    (periodic z)."""
    c = sim.cfg
    j, k = c.nx // 2, c.ny // 2
    ey = sim.get_field("Ey")
    bx = sim.get_field("Bx")
    nz = c.nz
    periodic = c.zbc == 0
    out = np.zeros(nz + 1)
    for i in range(nz + 1):
        ii = i % nz if periodic else i
        e = ey[ii, j, k] if ey.ndim == 3 else ey[ii, j]
        if frame == 0:
            out[i] = e
            continue
        def bxat(r):
            if periodic:
                r %= nz
            elif r < 0 or r > nz:
                return 0.0
            return bx[r, j, k] if bx.ndim == 3 else bx[r, j]
        b = 0.5 * (bxat(i - 1) + bxat(i))
        out[i] = gamma_b * (e - beta_of_gamma(gamma_b) * b)
    return out


def _along(rec_r: np.ndarray, z0: float, dz: float, zp: float) -> float:
    """Linear interpolation of one record at boosted position zp; NaN off it."""
    n = len(rec_r)
    u = (zp - z0) / dz
    if not (0.0 <= u <= n - 1):
        return math.nan
    i = min(int(math.floor(u)), n - 2)
    f = u - i
    return rec_r[i] + f * (rec_r[i + 1] - rec_r[i])


def back_transform(rec, t_prime, z0_prime, dz_prime, gamma_b, t0, dt, nt, zeta0, dzeta, nzeta,
                   v_window) -> np.ndarray:
    """Lab-frame values out[m, k] at t = t0 + m dt, zeta = zeta0 + k dzeta."""
    rec = np.asarray(rec, dtype=np.float64)
    tp_rec = np.asarray(t_prime, dtype=np.float64)
    z0 = np.asarray(z0_prime, dtype=np.float64)
    beta = beta_of_gamma(gamma_b)
    out = np.full((nt, nzeta), math.nan)
    for m in range(nt):
        t = t0 + m * dt
        for k in range(nzeta):
            z = zeta0 + k * dzeta + v_window * t
            tp = gamma_b * (t - beta * z)
            zp = gamma_b * (z - beta * t)
            if not (tp_rec[0] <= tp <= tp_rec[-1]):
                continue
            # the two records that bracket t'
            lo = max(r for r in range(len(tp_rec) - 1) if tp_rec[r] <= tp)
            hi = lo + 1
            a = _along(rec[lo], z0[lo], dz_prime, zp)
            b = _along(rec[hi], z0[hi], dz_prime, zp)
            out[m, k] = a + (tp - tp_rec[lo]) / (tp_rec[hi] - tp_rec[lo]) * (b - a)
    return out


def spectrum(rec, m: int) -> np.ndarray:
    """|X_q|^2, X_q = sum_i x_i exp(-2 pi i q i / m), q = 0..m/2, each record
    zero-padded to m points."""
    rec = np.atleast_2d(np.asarray(rec, dtype=np.float64))
    return np.abs(np.fft.rfft(rec, n=m, axis=1)) ** 2
