"""Radar geometry of the oracle (test infrastructure; see the package header).

Sensing functions, paper Sec. II eqs. (1)-(2): for receiver q and a point x
    R_q(x)   = |x - x_TX| + |x - x_RX,q|                 (bistatic range sum, m)
    w_q(x)   = unit(x - x_TX) + unit(x - x_RX,q)         (gradient of R_q)
    U_q(x,v) = <w_q(x), v>                               (bistatic range rate, m/s)
The paper scales them as r = (2B/c) R and u = (2 f0 Tc / c) U with atoms
exp(j 2 pi r m).  Read with the physical FMCW scaling instead (the paper's
factor 2 is the monostatic round trip, and m indexes samples), the sensed
parameters in cycles per sample / per chirp are
    f_r = B R / (c Ms),     f_d = f0 Tc U / c,
and on the zero-padded FFT grids (N_r = P Ms range bins, N_d = P Mc Doppler
bins) the continuous bin coordinates are
    t_r = f_r N_r = (B P / c) R,     t_d = f_d N_d = (f0 Tc P Mc / c) U.
unit(0) is taken as 0 (the paper is silent; the workloads never reach it).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Radar:
    f0: float
    bw: float
    tc: float
    c: float
    ms: int
    mc: int
    pad_r: int
    pad_d: int
    tx: np.ndarray      # (2,)
    rx: np.ndarray      # (K, 2)
    centered: int = 1

    @property
    def k(self) -> int:
        return int(self.rx.shape[0])

    @property
    def nr(self) -> int:
        return self.pad_r * self.ms

    @property
    def nd(self) -> int:
        return self.pad_d * self.mc


def radar_from_scene(sc) -> Radar:
    return Radar(f0=float(sc.f0), bw=float(sc.bw), tc=float(sc.tc), c=float(sc.c), ms=int(sc.ms),
                 mc=int(sc.mc), pad_r=int(sc.pad), pad_d=int(sc.pad), tx=np.asarray(sc.tx, np.float64),
                 rx=np.asarray(sc.rx, np.float64), centered=int(sc.centered))


def _unit(dx, dy):
    n = np.hypot(dx, dy)
    safe = np.where(n > 0, n, 1.0)
    return np.where(n > 0, dx / safe, 0.0), np.where(n > 0, dy / safe, 0.0), n


def sensing(radar: Radar, q: int, x, y):
    """R_q and w_q = grad R_q at points (x, y): eqs. (1)-(2) without their scale factors."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    ux, uy, n_tx = _unit(x - radar.tx[0], y - radar.tx[1])
    vx, vy, n_rx = _unit(x - radar.rx[q, 0], y - radar.rx[q, 1])
    return n_tx + n_rx, ux + vx, uy + vy


def sensed_freqs(radar: Radar, q: int, x, y, vx, vy):
    """(f_r, f_d): cycles per fast-time sample and cycles per chirp at (x, v) for receiver q."""
    rr, wx, wy = sensing(radar, q, x, y)
    rate = wx * np.asarray(vx, np.float64) + wy * np.asarray(vy, np.float64)
    fr = radar.bw * rr / (radar.c * radar.ms)
    fd = radar.f0 * radar.tc * rate / radar.c
    return fr, fd


def bin_coords(radar: Radar, q: int, x, y, vx, vy):
    """Continuous (range-bin, Doppler-bin) coordinates (t_r, t_d) on the zero-padded maps."""
    fr, fd = sensed_freqs(radar, q, x, y, vx, vy)
    return fr * radar.nr, fd * radar.nd


def grid_axis(lo: float, hi: float, n: int) -> np.ndarray:
    """Inclusive uniform axis of the grids X_G, V_G (Sec. III): lo + i (hi - lo)/(n - 1)."""
    if n == 1:
        return np.array([lo], dtype=np.float64)
    return lo + np.arange(n, dtype=np.float64) * ((hi - lo) / (n - 1))


def grid_axes(grid):
    return [grid_axis(grid.lo[a], grid.hi[a], grid.n[a]) for a in range(4)]


def grid_point(grid, index: int):
    """(x, y, vx, vy) of linear index ((ix*Ny + iy)*Nvx + ivx)*Nvy + ivy."""
    nx, ny, nvx, nvy = grid.n
    ivy = index % nvy
    ivx = (index // nvy) % nvx
    iy = (index // (nvy * nvx)) % ny
    ix = index // (nvy * nvx * ny)
    ax = grid_axes(grid)
    return np.array([ax[0][ix], ax[1][iy], ax[2][ivx], ax[3][ivy]])
