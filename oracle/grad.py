"""Gradients of the decisions at continuous points (test infrastructure; see the package header).

Not in the paper: for gradient-based refinement the decisions are needed at
continuous theta = (x, y, vx, vy), with derivatives with respect to theta
and to the receiver positions rx_q.

Direct decision, D_dir = sum_q |c_q|^2 with c_q = M_00 and the moments
M_pq = sum_{m,s} Y_q[m][s] E s^p m^q, E = exp(-j 2 pi (f_r s + f_d m)) (see
refine.py):
  dc_q/dp = -j 2 pi (df_r/dp M_10 + df_d/dp M_01),   dD/dp = 2 Re(conj(c_q) dc_q/dp).
Grid-hopping decision, D_gh = sum_q |I_q|^2 with the interpolated map value
I_q = sum_taps W(a - i) W(b - l) Z_q[i][l] (gh.py) at (t_r, t_d) = (N_r f_r, N_d f_d):
  dI/dt_r = sum W'(a - i) W(b - l) Z,   dI/dt_d = sum W(a - i) W'(b - l) Z,
  dD/dp = 2 Re(conj(I_q) (N_r dI/dt_r df_r/dp + N_d dI/dt_d df_d/dp)).
The bilinear weights (1 - f, f) have the piecewise-constant derivative
(-1, 1); the Keys weights are differentiable.

Frequency derivatives: with respect to theta as in refine.freq_derivs; with
respect to receiver q's position, from R_q = |x - tx| + |x - rx_q| and
U_q = <unit(x - tx) + unit(x - rx_q), v>:
  df_r/drx_q = -beta_r u,   df_d/drx_q = -beta_d (I - u u^T) v / rho,
with rho = |x - rx_q|, u = (x - rx_q) / rho.  Only receiver q's own
frequencies depend on rx_q.
"""
from __future__ import annotations

import numpy as np

from . import gh, maps, radar as rd, refine


def rx_freq_derivs(radar: rd.Radar, q: int, theta):
    """(df_r/drx_q, df_d/drx_q), each of shape (2,)."""
    p = np.asarray(theta[:2], np.float64)
    v = np.asarray(theta[2:], np.float64)
    beta_r = radar.bw / (radar.c * radar.ms)
    beta_d = radar.f0 * radar.tc / radar.c
    d = p - radar.rx[q]
    rho = float(np.hypot(d[0], d[1]))
    if rho == 0.0:
        return np.zeros(2), np.zeros(2)
    u = d / rho
    return -beta_r * u, -beta_d * ((np.eye(2) - np.outer(u, u)) @ v) / rho


def direct_value_grad(y: np.ndarray, radar: rd.Radar, theta):
    """(D_dir, dD/dtheta (4,), dD/drx (K, 2)) at theta."""
    theta = np.asarray(theta, np.float64)
    tp = 2.0 * np.pi
    dval = 0.0
    grad = np.zeros(4)
    grad_rx = np.zeros((radar.k, 2))
    for q in range(radar.k):
        fr, fd, gr, gd, _, _ = refine.freq_derivs(radar, q, theta)
        mo = refine.moments(y[q], fr, fd)
        c = mo[(0, 0)]
        dc = -1j * tp * (gr * mo[(1, 0)] + gd * mo[(0, 1)])
        dval += abs(c) ** 2
        grad += 2.0 * np.real(np.conj(c) * dc)
        rr, rd_ = rx_freq_derivs(radar, q, theta)
        dcx = -1j * tp * (rr * mo[(1, 0)] + rd_ * mo[(0, 1)])
        grad_rx[q] = 2.0 * np.real(np.conj(c) * dcx)
    return dval, grad, grad_rx


def keys_derivative(d):
    """dW/dd of the Keys kernel (a = -1/2) at signed offset d."""
    d = np.asarray(d, np.float64)
    x = np.abs(d)
    g_in = 4.5 * x ** 2 - 5.0 * x
    g_out = -1.5 * x ** 2 + 5.0 * x - 4.0
    return np.sign(d) * np.where(x <= 1.0, g_in, np.where(x < 2.0, g_out, 0.0))


def weights_and_derivs(t: float, kind: int):
    """Taps, weights and d(weight)/dt of the interpolation along one axis."""
    t0 = np.floor(t)
    f = t - t0
    if kind == gh.BILINEAR:
        offs = (0, 1)
        ws = (1.0 - f, f)
        dws = (-1.0, 1.0)
    else:
        offs = (-1, 0, 1, 2)
        ws = tuple(float(gh.keys_weight(f - o)) for o in offs)
        dws = tuple(float(keys_derivative(f - o)) for o in offs)
    return [int(t0) + o for o in offs], ws, dws


def interpolate_with_derivs(zq, tr: float, td: float, kind: int, ms: int, mc: int, centered: int):
    """(I, dI/dt_r, dI/dt_d) at one continuous map coordinate."""
    ri, rw, rdw = weights_and_derivs(tr, kind)
    di, dw, ddw = weights_and_derivs(td, kind)
    val = dr = dd = 0.0 + 0.0j
    for a in range(len(ri)):
        for b in range(len(di)):
            z = complex(maps.node_value(zq, ri[a], di[b], ms, mc, centered))
            val += rw[a] * dw[b] * z
            dr += rdw[a] * dw[b] * z
            dd += rw[a] * ddw[b] * z
    return val, dr, dd


def gh_value_grad(z: np.ndarray, radar: rd.Radar, theta, kind: int):
    """(D_gh, dD/dtheta (4,), dD/drx (K, 2)) at theta."""
    theta = np.asarray(theta, np.float64)
    dval = 0.0
    grad = np.zeros(4)
    grad_rx = np.zeros((radar.k, 2))
    for q in range(radar.k):
        fr, fd, gr, gd, _, _ = refine.freq_derivs(radar, q, theta)
        val, dtr, dtd = interpolate_with_derivs(z[q], fr * radar.nr, fd * radar.nd, kind, radar.ms, radar.mc,
                                                radar.centered)
        dval += abs(val) ** 2
        grad += 2.0 * np.real(np.conj(val) * (dtr * radar.nr * gr + dtd * radar.nd * gd))
        rr, rd_ = rx_freq_derivs(radar, q, theta)
        grad_rx[q] = 2.0 * np.real(np.conj(val) * (dtr * radar.nr * rr + dtd * radar.nd * rd_))
    return dval, grad, grad_rx
