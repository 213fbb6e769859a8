"""Direct decision of the oracle (test infrastructure; see the package header).

The direct method (paper Sec. I and Sec. III) maximises over the 4D grid the
energy of the scalar products between each receiver's frame and the model
atom of eq. (3):
    c_q(x, v) = <Y_q, b(f_d) (x) a(f_r)> = sum_m sum_s Y_q[m][s] exp(-j 2 pi (f_r s + f_d m))
    D_dir(x, v) = sum_q |c_q(x, v)|^2
with (f_r, f_d) = radar.sensed_freqs(q, x, v).  This is the joint location-
velocity objective; the paper's eqs. (5)-(6) factorise it into a location
search (energy over chirps, range atom only) followed by a velocity search.

c_q is the bilinear form b^H Y_q conj(a): it is evaluated as the matrix-vector
product g = Y_q conj(a) followed by the inner product with conj(b), which is
the definition itself, not a reordering.
"""
from __future__ import annotations

import numpy as np

from . import radar as rd


def range_atom(fr, ms: int):
    """a(f_r) of eq. (3): a_s = exp(j 2 pi f_r s)."""
    return np.exp(2j * np.pi * np.asarray(fr, np.float64)[..., None] * np.arange(ms))


def doppler_atom(fd, mc: int):
    """b(f_d) of eq. (3): b_m = exp(j 2 pi f_d m)."""
    return np.exp(2j * np.pi * np.asarray(fd, np.float64)[..., None] * np.arange(mc))


def correlation(yq: np.ndarray, fr, fd):
    """<Y_q, b(f_d) (x) a(f_r)> for arrays of (f_r, f_d) of equal shape."""
    yq = np.asarray(yq).astype(np.complex128)
    fr = np.asarray(fr, np.float64)
    fd = np.asarray(fd, np.float64)
    g = np.conj(range_atom(fr, yq.shape[1])) @ yq.T          # (..., Mc): sum_s Y[m][s] conj(a_s)
    return np.sum(g * np.conj(doppler_atom(fd, yq.shape[0])), axis=-1)


def direct_points(y: np.ndarray, radar: rd.Radar, x, y_, vx, vy):
    """D_dir at arbitrary points (arrays of equal shape)."""
    x, y_, vx, vy = np.broadcast_arrays(*(np.asarray(a, np.float64) for a in (x, y_, vx, vy)))
    d = np.zeros(x.shape)
    for q in range(radar.k):
        fr, fd = rd.sensed_freqs(radar, q, x, y_, vx, vy)
        d += np.abs(correlation(y[q], fr.ravel(), fd.ravel())).reshape(x.shape) ** 2
    return d


def location_energy(y: np.ndarray, radar: rd.Radar, x, y_):
    """Eq. (5)'s objective: sum_q sum_m |<Y_q[m], a(f_r,q(x))>|^2 at location(s) (x, y)."""
    x, y_ = np.broadcast_arrays(np.asarray(x, np.float64), np.asarray(y_, np.float64))
    e = np.zeros(x.shape)
    for q in range(radar.k):
        fr, _ = rd.sensed_freqs(radar, q, x, y_, 0.0, 0.0)
        g = np.conj(range_atom(fr.ravel(), radar.ms)) @ np.asarray(y[q]).astype(np.complex128).T
        e += np.sum(np.abs(g) ** 2, axis=-1).reshape(x.shape)
    return e


def direct_decision(y: np.ndarray, radar: rd.Radar, grid) -> np.ndarray:
    """D_dir over the whole grid, shape (Nx, Ny, Nvx, Nvy)."""
    ax = rd.grid_axes(grid)
    nx, ny, nvx, nvy = grid.n
    vxx, vyy = np.meshgrid(ax[2], ax[3], indexing="ij")
    out = np.zeros((nx, ny, nvx, nvy))
    yc = np.asarray(y).astype(np.complex128)
    for q in range(radar.k):
        for ix in range(nx):
            for iy in range(ny):
                fr, fd = rd.sensed_freqs(radar, q, ax[0][ix], ax[1][iy], vxx, vyy)
                g = yc[q] @ np.conj(range_atom(fr, radar.ms))              # (Mc,)
                c = np.conj(doppler_atom(fd, radar.mc)) @ g               # (Nvx, Nvy)
                out[ix, iy] += np.abs(c) ** 2
    return out
