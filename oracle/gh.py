"""Grid-hopping decision of the oracle (test infrastructure; see the package header).

Paper Sec. IV, eq. (7): the scalar product of a receiver's data with the atom
of a grid point is approximated by a weighted sum c^T z_I of FFT outputs over
an index set I.  Here the index set and weights are those of separable
interpolation of the 2D map at the continuous bin coordinates (t_r, t_d)
of the grid point (radar.bin_coords):
  bilinear : taps {0, 1} on each axis, weights (1 - f, f)
  bicubic  : taps {-1, 0, 1, 2} on each axis, Keys cubic-convolution weights
             W(f - tap) with parameter a = -1/2
with f the fractional part of the coordinate.  Taps outside one period use
maps.node_value (periodic, with the centring sign).  The decision is the
noncoherent sum over receivers, D(x, v) = sum_q |I_q(x, v)|^2, as the direct
method's objective sums |<Y_q, atom>|^2 over q (eqs. (5)-(6)).

The paper's own choice (polar interpolation in range, nearest neighbour in
Doppler) is a different index-set/weight rule, used with the factorised
decisions of eqs. (5)-(6) in factor.py; the joint 4D decision here uses
bilinear and bicubic interpolation.
"""
from __future__ import annotations

import numpy as np

from . import maps, radar as rd

BILINEAR, BICUBIC = 0, 1


def keys_weight(d):
    """Keys cubic convolution kernel, a = -1/2."""
    d = np.abs(np.asarray(d, np.float64))
    w_in = 1.5 * d ** 3 - 2.5 * d ** 2 + 1.0
    w_out = -0.5 * d ** 3 + 2.5 * d ** 2 - 4.0 * d + 2.0
    return np.where(d <= 1.0, w_in, np.where(d < 2.0, w_out, 0.0))


def taps_and_weights(t, kind: int):
    """Integer tap positions and weights for continuous coordinate t (arrays broadcast)."""
    t = np.asarray(t, np.float64)
    t0 = np.floor(t)
    f = t - t0
    if kind == BILINEAR:
        offs = (0, 1)
        ws = (1.0 - f, f)
    elif kind == BICUBIC:
        offs = (-1, 0, 1, 2)
        ws = tuple(keys_weight(f - o) for o in offs)
    else:
        raise ValueError("unknown interpolation kind")
    return [(t0 + o).astype(np.int64) for o in offs], list(ws)


def interpolate(zq: np.ndarray, tr, td, kind: int, ms: int, mc: int, centered: int):
    """Interpolated map value at continuous (t_r, t_d): the right-hand side of eq. (7)."""
    ri, rw = taps_and_weights(tr, kind)
    di, dw = taps_and_weights(td, kind)
    acc = np.zeros(np.broadcast(np.asarray(tr), np.asarray(td)).shape, dtype=np.complex128)
    for a in range(len(ri)):
        for b in range(len(di)):
            acc = acc + rw[a] * dw[b] * maps.node_value(zq, ri[a], di[b], ms, mc, centered)
    return acc


def gh_points(z: np.ndarray, radar: rd.Radar, x, y, vx, vy, kind: int):
    """D_gh at arbitrary points (arrays of equal shape)."""
    d = 0.0
    for q in range(radar.k):
        tr, td = rd.bin_coords(radar, q, x, y, vx, vy)
        d = d + np.abs(interpolate(z[q], tr, td, kind, radar.ms, radar.mc, radar.centered)) ** 2
    return d


def gh_decision(z: np.ndarray, radar: rd.Radar, grid, kind: int) -> np.ndarray:
    """D_gh over the whole grid, shape (Nx, Ny, Nvx, Nvy)."""
    ax = rd.grid_axes(grid)
    nx, ny, nvx, nvy = grid.n
    out = np.empty((nx, ny, nvx, nvy), dtype=np.float64)
    yy, vxx, vyy = np.meshgrid(ax[1], ax[2], ax[3], indexing="ij")
    for ix in range(nx):
        out[ix] = gh_points(z, radar, np.full_like(yy, ax[0][ix]), yy, vxx, vyy, kind)
    return out
