"""Factorised decisions of the oracle (test infrastructure; see the package header).

Paper Sec. III, eqs. (5)-(6).  The direct method as the paper runs it first
estimates the location from the energy of the per-chirp range correlations,
    E(x) = sum_q sum_m |<Y_q[m], a(f_r,q(x))>|^2,          x^ = argmax over X_G   (5)
then the velocity at x^ from the chirp sequence of range correlations there,
g_q[m] = <Y_q[m], a(f_r,q(x^))>,
    V(v) = sum_q |<g_q, b(f_d,q(x^, v))>|^2,                v^ = argmax over V_G   (6)
(reading: the atom of (6) is the Doppler atom b, since f_d is in cycles per
chirp; V(v) is then the joint decision D_dir(x^, v)).

Grid hopping (Sec. IV) replaces the scalar products of (5) by c^T z_I, an
interpolation of each chirp's zero-padded range FFT z, and those of (6) by a
single FFT bin (nearest neighbour) of the zero-padded FFT over chirps of the
interpolated sequence g_q.  The range rule the paper uses is polar
interpolation (the three-atom circle approximation of the continuous basis
pursuit work it cites): the atoms at bin offsets tau = -1, 0, 1 from the
nearest bin i lie on a circle in the real vector space C^Ms = R^(2 Ms),
    f(tau) ~ C + R (cos(theta tau) U + sin(theta tau) V),   U, V orthonormal,
whose angle per bin, theta, follows from the chord lengths:
    |f(1) - f(-1)|^2 / |f(1) - f(0)|^2 = 2 (1 + cos theta),
    |f(a) - f(b)|^2 = 2 Ms - 2 Re <f(a), f(b)>.
Solving for C, R U, R V through the three atoms and taking the scalar product
with the data gives
    <y, f(tau)> ~ w_-1 z_{i-1} + w_0 z_i + w_1 z_{i+1},
    w_0 = 1 + 2A,  w_+-1 = -A +- B,
    A = (cos(theta tau) - 1) / (2 (1 - cos theta)),  B = sin(theta tau) / (2 sin theta),
with tau = t_r - i in [-1/2, 1/2].  Bilinear and Keys bicubic range rules
(gh.taps_and_weights) are also provided.  Taps outside one period wrap with
the centring sign, as in maps.node_value.
"""
from __future__ import annotations

import numpy as np

from . import direct, gh, maps, peaks, radar as rd

BILINEAR, BICUBIC, POLAR = 0, 1, 2


def range_spectra(y: np.ndarray, pad_r: int, centered: int) -> np.ndarray:
    """z[q][m][i] = sum_s Y_q[m][s] exp(-j 2 pi i (s - c_s) / N_r), i < N_r = P Ms (library FFT + shift)."""
    y = np.asarray(y).astype(np.complex128)
    ms = y.shape[-1]
    nr = pad_r * ms
    z = np.fft.fft(y, n=nr, axis=-1)
    if centered:
        z = z * np.exp(2j * np.pi * np.arange(nr) * ((ms - 1) / 2.0) / nr)
    return z


def atom_inner(ms: int, nr: int, centered: int, d: float) -> float:
    """Re <f(tau), f(tau + d)> for the range atoms of the FFT grid (d in bins), by its sum."""
    s = np.arange(ms, dtype=np.float64)
    c = (ms - 1) / 2.0 if centered else 0.0
    return float(np.real(np.sum(np.exp(-2j * np.pi * d * (s - c) / nr))))


def polar_theta(ms: int, pad_r: int, centered: int) -> float:
    """Circle angle per bin of the polar rule, from the chord-length ratio."""
    nr = pad_r * ms
    h1 = ms - atom_inner(ms, nr, centered, 1.0)     # |f(0) - f(1)|^2 / 2
    h2 = ms - atom_inner(ms, nr, centered, 2.0)     # |f(-1) - f(1)|^2 / 2
    return float(np.arccos(h2 / (2.0 * h1) - 1.0))


def polar_weights(tau, theta: float):
    """Weights of taps -1, 0, +1 around the nearest bin for offsets tau (arrays)."""
    tau = np.asarray(tau, np.float64)
    a = (np.cos(theta * tau) - 1.0) / (2.0 * (1.0 - np.cos(theta)))
    b = np.sin(theta * tau) / (2.0 * np.sin(theta))
    return -a - b, 1.0 + 2.0 * a, -a + b


def range_taps(t, kind: int, theta: float | None = None):
    """Integer range taps and weights at continuous bin coordinate(s) t."""
    t = np.asarray(t, np.float64)
    if kind == POLAR:
        i = np.floor(t + 0.5)
        return [(i + o).astype(np.int64) for o in (-1, 0, 1)], list(polar_weights(t - i, theta))
    return gh.taps_and_weights(t, kind)


def chirp_values(zq: np.ndarray, tr: float, kind: int, ms: int, centered: int, theta: float | None):
    """The interpolated range correlation of every chirp of one receiver at t_r: [Mc] complex."""
    nr = zq.shape[-1]
    taps, ws = range_taps(tr, kind, theta)
    sign = maps.wrap_sign(ms, centered)
    acc = np.zeros(zq.shape[0], dtype=np.complex128)
    for i, w in zip(taps, ws):
        wraps, ii = divmod(int(i), nr)
        acc = acc + float(w) * zq[:, ii] * sign ** wraps
    return acc


def _theta(radar: rd.Radar, kind: int):
    return polar_theta(radar.ms, radar.pad_r, radar.centered) if kind == POLAR else None


def gh_location_energy(zr: np.ndarray, radar: rd.Radar, grid, kind: int) -> np.ndarray:
    """Eq. (5) with its scalar products interpolated from the range spectra zr[q][m][i]: [Nx][Ny]."""
    ax = rd.grid_axes(grid)
    theta = _theta(radar, kind)
    out = np.zeros((grid.n[0], grid.n[1]))
    for ix in range(grid.n[0]):
        for iy in range(grid.n[1]):
            for q in range(radar.k):
                tr, _ = rd.bin_coords(radar, q, ax[0][ix], ax[1][iy], 0.0, 0.0)
                g = chirp_values(zr[q], float(tr), kind, radar.ms, radar.centered, theta)
                out[ix, iy] += float(np.sum(np.abs(g) ** 2))
    return out


def direct_location_energy(y: np.ndarray, radar: rd.Radar, grid) -> np.ndarray:
    """Eq. (5)'s objective over the location grid: [Nx][Ny]."""
    ax = rd.grid_axes(grid)
    xx, yy = np.meshgrid(ax[0], ax[1], indexing="ij")
    return direct.location_energy(y, radar, xx, yy)


def gh_velocity(zr: np.ndarray, radar: rd.Radar, grid, loc: int, kind: int) -> np.ndarray:
    """Eq. (6) by grid hopping at location index loc: each receiver's interpolated chirp
    sequence g_q, its zero-padded (centred) FFT over chirps G_q, and the nearest bin
    round(t_d) of G_q for every velocity: [Nvx][Nvy]."""
    ax = rd.grid_axes(grid)
    ix, iy = divmod(int(loc), grid.n[1])
    x, y_ = ax[0][ix], ax[1][iy]
    theta = _theta(radar, kind)
    vxx, vyy = np.meshgrid(ax[2], ax[3], indexing="ij")
    nd = radar.nd
    out = np.zeros(vxx.shape)
    for q in range(radar.k):
        tr, _ = rd.bin_coords(radar, q, x, y_, 0.0, 0.0)
        g = chirp_values(zr[q], float(tr), kind, radar.ms, radar.centered, theta)
        gq = np.fft.fft(g, n=nd)
        if radar.centered:
            gq = gq * np.exp(2j * np.pi * np.arange(nd) * ((radar.mc - 1) / 2.0) / nd)
        _, td = rd.bin_coords(radar, q, x, y_, vxx, vyy)
        l = np.floor(td + 0.5).astype(np.int64) % nd
        out += np.abs(gq[l]) ** 2          # a whole-period wrap only changes the sign
    return out


def direct_velocity(y: np.ndarray, radar: rd.Radar, grid, loc: int) -> np.ndarray:
    """Eq. (6) exactly: the joint decision at location index loc over the velocity grid."""
    ax = rd.grid_axes(grid)
    ix, iy = divmod(int(loc), grid.n[1])
    vxx, vyy = np.meshgrid(ax[2], ax[3], indexing="ij")
    return direct.direct_points(y, radar, np.full_like(vxx, ax[0][ix]), np.full_like(vxx, ax[1][iy]), vxx, vyy)


def factored_estimate(loc_energy: np.ndarray, velocity_at):
    """(location index, velocity index, linear 4D grid index, V(v^), V slab) of eqs. (5)-(6):
    the first maximum of the location energy, then of the velocity decision there."""
    _, il = peaks.first_max(np.asarray(loc_energy).ravel())
    vel = velocity_at(il)
    vv, iv = peaks.first_max(vel.ravel())
    return il, iv, il * vel.size + iv, vv, vel
