"""Off-grid refinement of the direct decision (test infrastructure; see the package header).

Not in the paper: the grid estimators stop at a grid cell.  The refinement
maximises the exact direct decision D(theta) = sum_q |c_q(theta)|^2 (see
direct.py) over continuous theta = (x, y, vx, vy) within one grid cell of a
starting cell, by Newton ascent with analytic derivatives.

Derivatives, for receiver q with legs d_1 = x - x_TX, d_2 = x - x_RX,q,
rho_i = |d_i|, u_i = d_i / rho_i (eqs. (1)-(2)):
  f_r = beta_r R,  beta_r = B/(c Ms);    f_d = beta_d <w, v>,  beta_d = f0 Tc / c
  d f_r / d x = beta_r w,                 d f_d / d v = beta_d w
  d f_d / d x = beta_d J v,               J = sum_i (I - u_i u_i^T) / rho_i
  d2 f_r / dx dx = beta_r J,              d2 f_d / dx dv = beta_d J
  d2 f_d / dx_a dx_b = -beta_d sum_i [u_b v_a + u_a v_b + (u.v)(delta_ab - 3 u_a u_b)] / rho_i^2
With E = exp(-j 2 pi (f_r s + f_d m)) and the moments
  M_pq = sum_{m,s} Y[m][s] E s^p m^q,
  c = M_00,  dc/da = -j 2 pi (f_r,a M_10 + f_d,a M_01),
  d2c/da db = -4 pi^2 (f_r,a f_r,b M_20 + (f_r,a f_d,b + f_d,a f_r,b) M_11 + f_d,a f_d,b M_02)
              - j 2 pi (f_r,ab M_10 + f_d,ab M_01),
  dD/da = 2 Re(conj(c) dc/da),  d2D/da db = 2 Re(conj(dc/db) dc/da + conj(c) d2c/da db).

The refined estimate is the converged local maximiser of D over the box
|theta_a - theta_0,a| <= h_a (one grid step per axis) reached by ascent from
the starting cell theta_0: the point where the box-projected Newton step
vanishes (KKT stationarity on the box), found with a generous budget so that
the answer does not depend on how the search is tuned.  Coordinates
z = (theta - theta_0) / h; an axis with a single grid point (h = 0) is held.
One iteration, a projected Newton step for the bound-constrained maximum
(Bertsekas' projected Newton method, with an epsilon-active set):
  w     = max_a |clamp(z_a + g_a / L) - z_a|, L the largest |diagonal entry|
          of the Hessian in z (how far z is from stationary, in cells);
  eps   = min(EPS_ACTIVE, w);
  push  = the coordinates within eps of a face of the box whose gradient
          component points out of it: their step is one cell outwards, so
          the projection puts them on the face;
  step  = on the other free coordinates, sum_i (e_i . g) /
          max(|lambda_i|, 1e-12 max|lambda|) e_i over the eigenpairs of the
          Hessian in z restricted to them (the Newton step of the reduced
          problem where its Hessian is negative definite, an ascent direction
          everywhere);
  converged when the projected step clamp(z + step) - z is below `tol`
          cells in every coordinate (the reduced gradient vanishes and every
          pushed coordinate is on its face: KKT on the box);
  candidate = clamp(z + step, [-1, 1]); while D(candidate) < D(z), halve the
          step (up to `max_halvings` times); move to the candidate;
  converged also when the accepted move is below `tol` cells (z is then
          stationary to the precision of D).
The loop runs at most `max_iter` iterations; refine_one reports whether it
converged (a search that finds no ascent within `max_halvings` halvings, or
runs out of iterations, is reported as not converged).
"""
from __future__ import annotations

import numpy as np

from . import radar as rd

ORDER = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]   # (p, q) of the moments M_pq
EPS_ACTIVE = 1e-2     # cells: the widest band next to a face in which an outward-pushed coordinate is put on it


def moments(yq: np.ndarray, fr: float, fd: float) -> dict:
    yq = np.asarray(yq).astype(np.complex128)
    mc, ms = yq.shape
    s = np.arange(ms, dtype=np.float64)[None, :]
    m = np.arange(mc, dtype=np.float64)[:, None]
    ye = yq * np.exp(-2j * np.pi * (fr * s + fd * m))
    return {(p, q): complex(np.sum(ye * s ** p * m ** q)) for (p, q) in ORDER}


def freq_derivs(radar: rd.Radar, q: int, theta):
    """(f_r, f_d, grad f_r (4), grad f_d (4), hess f_r (4x4), hess f_d (4x4))."""
    p = np.asarray(theta[:2], np.float64)
    v = np.asarray(theta[2:], np.float64)
    beta_r = radar.bw / (radar.c * radar.ms)
    beta_d = radar.f0 * radar.tc / radar.c
    w = np.zeros(2)
    jac = np.zeros((2, 2))
    hxx = np.zeros((2, 2))
    rsum = 0.0
    for anchor in (radar.tx, radar.rx[q]):
        d = p - anchor
        rho = float(np.hypot(d[0], d[1]))
        if rho == 0.0:
            continue
        u = d / rho
        rsum += rho
        w += u
        jac += (np.eye(2) - np.outer(u, u)) / rho
        uv = float(u @ v)
        hxx -= (np.outer(v, u) + np.outer(u, v) + uv * (np.eye(2) - 3.0 * np.outer(u, u))) / rho ** 2
    fr = beta_r * rsum
    fd = beta_d * float(w @ v)
    gr = np.concatenate([beta_r * w, np.zeros(2)])
    gd = np.concatenate([beta_d * (jac @ v), beta_d * w])
    hr = np.zeros((4, 4))
    hr[:2, :2] = beta_r * jac
    hd = np.zeros((4, 4))
    hd[:2, :2] = beta_d * hxx
    hd[:2, 2:] = beta_d * jac
    hd[2:, :2] = beta_d * jac.T
    return fr, fd, gr, gd, hr, hd


def decision_derivs(y: np.ndarray, radar: rd.Radar, theta):
    """(D, gradient (4), Hessian (4x4)) of the direct decision at theta."""
    dval = 0.0
    grad = np.zeros(4)
    hess = np.zeros((4, 4))
    tp = 2.0 * np.pi
    for q in range(radar.k):
        fr, fd, gr, gd, hr, hd = freq_derivs(radar, q, theta)
        mo = moments(y[q], fr, fd)
        c = mo[(0, 0)]
        dc = -1j * tp * (gr * mo[(1, 0)] + gd * mo[(0, 1)])
        d2c = (-tp * tp * (np.outer(gr, gr) * mo[(2, 0)] + (np.outer(gr, gd) + np.outer(gd, gr)) * mo[(1, 1)]
                           + np.outer(gd, gd) * mo[(0, 2)])
               - 1j * tp * (hr * mo[(1, 0)] + hd * mo[(0, 1)]))
        dval += abs(c) ** 2
        grad += 2.0 * np.real(np.conj(c) * dc)
        hess += 2.0 * np.real(np.outer(dc, np.conj(dc)) + np.conj(c) * d2c)
    return dval, grad, hess


def decision_value(y, radar, theta) -> float:
    total = 0.0
    for q in range(radar.k):
        fr, fd, *_ = freq_derivs(radar, q, theta)
        total += abs(moments(y[q], fr, fd)[(0, 0)]) ** 2
    return total


def grid_steps(grid) -> np.ndarray:
    return np.array([0.0 if grid.n[a] == 1 else (grid.hi[a] - grid.lo[a]) / (grid.n[a] - 1) for a in range(4)])


def refine_one(y, radar: rd.Radar, theta0, h, max_iter: int = 200, tol: float = 1e-10,
               max_halvings: int = 60, report: bool = False):
    """Converged local maximiser of D within one grid step of theta0 (see the module header)."""
    theta0 = np.asarray(theta0, np.float64)
    z = np.zeros(4)
    free = h > 0
    d_cur = decision_value(y, radar, theta0)
    converged = False
    iters = 0
    for iters in range(1, max_iter + 1):
        _, g, hth = decision_derivs(y, radar, theta0 + z * h)
        gz = np.where(free, g * h, 0.0)
        hz = hth * np.outer(h, h)
        curv = max(float(np.max(np.abs(np.diag(hz)[free]))) if free.any() else 0.0, 1e-300)
        w = float(np.max(np.abs(np.clip(z + gz / curv, -1.0, 1.0) - z)))
        eps = min(EPS_ACTIVE, w)
        push = free & (((z >= 1.0 - eps) & (gz > 0.0)) | ((z <= -1.0 + eps) & (gz < 0.0)))
        mov = free & ~push
        step = np.where(push, np.sign(gz), 0.0)
        if mov.any():
            lam, vec = np.linalg.eigh(hz[np.ix_(mov, mov)])
            floor = 1e-12 * max(np.max(np.abs(lam)), 1e-300)
            step[mov] = vec @ ((vec.T @ gz[mov]) / np.maximum(np.abs(lam), floor))
        if float(np.max(np.abs(np.clip(z + step, -1.0, 1.0) - z))) < tol:
            converged = True
            break
        accepted = False
        for _ in range(max_halvings + 1):
            cand = np.clip(z + step, -1.0, 1.0)
            d_new = decision_value(y, radar, theta0 + cand * h)
            if d_new >= d_cur:
                accepted = True
                break
            step = step * 0.5
        if not accepted:
            break
        move = float(np.max(np.abs(cand - z)))
        z, d_cur = cand, d_new
        if move < tol:
            converged = True
            break
    theta = theta0 + z * h
    return (theta, converged, iters) if report else theta


def refine(y, radar: rd.Radar, grid, cells, max_iter: int = 200, tol: float = 1e-10, report: bool = False):
    """Refined (x, y, vx, vy) for each starting cell (linear grid index); with
    `report`, also whether each converged and its iteration count."""
    h = grid_steps(grid)
    res = [refine_one(y, radar, rd.grid_point(grid, int(c)), h, max_iter, tol, report=True) for c in cells]
    theta = np.stack([r[0] for r in res])
    if report:
        return theta, np.array([r[1] for r in res]), np.array([r[2] for r in res])
    return theta
