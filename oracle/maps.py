"""Range-Doppler maps of the oracle (test infrastructure; see the package header).

Paper Sec. III (indirect method) and Sec. IV: the 2D FFT of each receiver's
frame; entry i of the FFT along fast time is the correlation of a chirp with
the range atom a(r_i) at the i-th frequency of the FFT grid.  With zero
padding by P on both axes (zeros appended, rectangular window) the map of
receiver q is, by definition,
    Z_q[i][l] = sum_{m<Mc} sum_{s<Ms} Y_q[m][s] exp(-j 2 pi (i (s - c_s)/N_r + l (m - c_m)/N_d))
for i < N_r = P Ms, l < N_d = P Mc.  Uncentred maps use c_s = c_m = 0;
centred maps use the centred atom index c_s = (Ms-1)/2, c_m = (Mc-1)/2, which
makes the correlation kernel real (a reading of the paper's remark that the
interpolation method must suit Fourier atoms; |Z| at the nodes is unchanged).
The scalar product is <u, v> = sum u conj(v), so maps are forward DFTs.

The FFT is used as a library step; the centring is the shift theorem applied
to its output.
"""
from __future__ import annotations

import numpy as np


def rd_maps(y: np.ndarray, pad_r: int, pad_d: int, centered: int) -> np.ndarray:
    """Z[q][i][l] (range bin i, Doppler bin l) from Y[q][m][s], complex128."""
    y = np.asarray(y).astype(np.complex128)
    _, mc, ms = y.shape
    nr, nd = pad_r * ms, pad_d * mc
    z = np.fft.fft2(y, s=(nd, nr), axes=(1, 2)).transpose(0, 2, 1)
    if centered:
        i = np.arange(nr)[:, None]
        l = np.arange(nd)[None, :]
        z = z * np.exp(2j * np.pi * (i * ((ms - 1) / 2.0) / nr + l * ((mc - 1) / 2.0) / nd))
    return np.ascontiguousarray(z)


def wrap_sign(m: int, centered: int) -> float:
    """Factor picked up by the (centred) correlation when its frequency grows by one cycle.

    C(f + 1) = exp(j 2 pi c) C(f) with c = (M-1)/2 for centred atoms, so the
    factor is (-1)^(M-1); uncentred correlations are 1-periodic.
    """
    return float((-1) ** (m - 1)) if centered else 1.0


def node_value(zq: np.ndarray, i, l, ms: int, mc: int, centered: int):
    """Correlation at integer bin indices (i, l) of any sign or size, from one map zq[N_r][N_d].

    The map holds one period; the value at i + a N_r, l + b N_d is the stored
    value times wrap_sign^a (range) and wrap_sign^b (Doppler).
    """
    nr, nd = zq.shape
    i = np.asarray(i, np.int64)
    l = np.asarray(l, np.int64)
    wi, ii = np.divmod(i, nr)
    wl, ll = np.divmod(l, nd)
    sr, sd = wrap_sign(ms, centered), wrap_sign(mc, centered)
    return zq[ii, ll] * np.power(sr, wi) * np.power(sd, wl)
